// gradient.hip -- gfx950 kernels of the gradient pre-processing (Introduction:
// smooth the image minimally, then take the gradient magnitude; both optional
// before Step I per the PRUF pipeline figure).
//
// float32 throughout. Per pixel the summation order is fixed (taps from -r to
// +r, x pass before y pass before z pass; Sobel terms in a fixed order), so
// the result does not depend on the launch configuration or on which other
// images are processed alongside.
//
// 2D images run one fused kernel per tile: the raw tile with its halo is staged
// in LDS, blurred along x, then along y, then the Sobel magnitude is taken, so
// the float image is read once and only the magnitude is written. 3D volumes
// use separable passes. Every workgroup stores its maximum in its own word (no
// atomics: same-line atomics from thousands of workgroups serialise), a small
// reduction takes the global maximum, and the quantiser reads that one word.
#include "ws_device.h"
#include "ws_kernels.h"

namespace wsk {

__device__ __forceinline__ int reflect_idx(int i, int n) {
    // half-sample symmetric borders: ... c b a | a b c ... (period 2n)
    if (i >= 0 && i < n) return i;
    int m = 2 * n;
    i %= m;
    if (i < 0) i += m;
    return i < n ? i : m - 1 - i;
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Block maximum, stored in part[blockIdx.x].
__device__ __forceinline__ void block_max_store(float m, float *part) {
    __shared__ float wmax[NTHREADS / 64];
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    if (__lane_id() == 0) wmax[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        float b = wmax[0];
        for (int w = 1; w < NTHREADS / 64; ++w) b = fmaxf(b, wmax[w]);
        part[blockIdx.x] = b;
    }
}

// out[b] = max of block b's share of in[0, n) (contiguous shares).
__global__ __launch_bounds__(NTHREADS) void k_grad_max(int32_t n, const float *__restrict__ in, float *__restrict__ out) {
    constexpr int U = 16;
    int32_t per = (n + (int32_t)gridDim.x - 1) / (int32_t)gridDim.x;
    int32_t lo = blockIdx.x * per, hi = lo + per < n ? lo + per : n;
    float m = 0.f;
    for (int32_t b = lo; b < hi; b += NTHREADS * U) {
        float v[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            int32_t i = b + j * NTHREADS + threadIdx.x;
            v[j] = i < hi ? in[i] : 0.f;
        }
#pragma unroll
        for (int j = 0; j < U; ++j) m = fmaxf(m, v[j]);
    }
    block_max_store(m, out);
}

// ---------------------------------------------------------------------------
// Fused 2D gradient: tile of GX x GY magnitudes per workgroup.
// LDS: raw (GY+2+2RB) x (GX+2+2RB), x-blurred (GY+2+2RB) x (GX+2), blurred
// (GY+2) x (GX+2); virtual coordinates outside the image are mirrored for the
// blur; the Sobel stencil clamps to the image (replicated border).
//
// Everything is sized by the compile-time radius RB: the host pads the taps
// of a smaller radius r with zeros (fma(0, x, s) == s for finite x, so the
// sums are those of the 2r+1 taps). Tiles whose halo lies inside the image
// (workgroup-uniform test) skip the mirroring and the clamping.
// ---------------------------------------------------------------------------
constexpr int GX = 64, GY = 16;

template <int RB>
__global__ __launch_bounds__(NTHREADS) void k_grad_fused2d(Geom g, const float *__restrict__ img,
                                                           float *__restrict__ mag, float *__restrict__ part,
                                                           BlurTaps taps) {
    constexpr int RW = GX + 2 + 2 * RB, RH = GY + 2 + 2 * RB;  // raw
    constexpr int BW = GX + 2, BH = GY + 2;                    // blurred
    constexpr int NT = 2 * RB + 1;
    __shared__ float raw[RW * RH];
    __shared__ float bx[BW * RH];
    __shared__ float bb[BW * BH];
    float w[NT];
#pragma unroll
    for (int k = 0; k < NT; ++k) w[k] = taps.w[k];
    const int tiles_x = (g.nx + GX - 1) / GX;
    const int t = xcd_tile(blockIdx.x, tiles_x * ((g.ny + GY - 1) / GY));
    const int x0 = (t % tiles_x) * GX, y0 = (t / tiles_x) * GY;
    const bool inside = x0 - 1 - RB >= 0 && x0 + GX + RB < g.nx && y0 - 1 - RB >= 0 && y0 + GY + RB < g.ny;
    {
        // batched raw loads: addresses first, then all loads, then LDS
        constexpr int CELLS = RW * RH;
        constexpr int PER = (CELLS + NTHREADS - 1) / NTHREADS;
        int32_t idx[PER];
        float v[PER];
        if (inside) {
            const int32_t b0 = (y0 - 1 - RB) * g.nx + (x0 - 1 - RB);
#pragma unroll
            for (int j = 0; j < PER; ++j) {
                int c = threadIdx.x + j * NTHREADS;
                idx[j] = c < CELLS ? b0 + (c / RW) * g.nx + c % RW : b0;
            }
        } else {
#pragma unroll
            for (int j = 0; j < PER; ++j) {
                int c = threadIdx.x + j * NTHREADS;
                int gx = reflect_idx(x0 - 1 - RB + c % RW, g.nx), gy = reflect_idx(y0 - 1 - RB + c / RW, g.ny);
                idx[j] = c < CELLS ? gx + gy * g.nx : 0;
            }
        }
#pragma unroll
        for (int j = 0; j < PER; ++j) v[j] = img[idx[j]];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            int c = threadIdx.x + j * NTHREADS;
            if (c < CELLS) raw[c] = v[j];
        }
    }
    __syncthreads();
    for (int c = threadIdx.x; c < BW * RH; c += NTHREADS) {
        const float *row = raw + (c / BW) * RW + c % BW;  // virtual x = x0-1+i-RB+k at row[k]
        float s = 0.f;
#pragma unroll
        for (int k = 0; k < NT; ++k) s = __fmaf_rn(w[k], row[k], s);
        bx[c] = s;
    }
    __syncthreads();
    for (int c = threadIdx.x; c < BW * BH; c += NTHREADS) {
        const float *col = bx + c;  // rows j .. j+2RB of column i
        float s = 0.f;
#pragma unroll
        for (int k = 0; k < NT; ++k) s = __fmaf_rn(w[k], col[k * BW], s);
        bb[c] = s;
    }
    __syncthreads();
    float m = 0.f;
    constexpr int PP = GX * GY / NTHREADS;
#pragma unroll
    for (int q = 0; q < PP; ++q) {
        const int c = threadIdx.x + q * NTHREADS;
        const int i = c % GX, j = c / GX;
        const int gx = x0 + i, gy = y0 + j;
        // local columns/rows of the neighbours (+1 for the ring), clamped to
        // the image at its border
        int xm = i, xp = i + 2, ym = j, yp = j + 2;
        if (!inside) {
            if (gx >= g.nx || gy >= g.ny) continue;
            xm = clampi(gx - 1, 0, g.nx - 1) - x0 + 1;
            xp = clampi(gx + 1, 0, g.nx - 1) - x0 + 1;
            ym = clampi(gy - 1, 0, g.ny - 1) - y0 + 1;
            yp = clampi(gy + 1, 0, g.ny - 1) - y0 + 1;
        }
        const int xc = i + 1, yc = j + 1;
        const float *r0 = bb + ym * BW, *r1 = bb + yc * BW, *r2 = bb + yp * BW;
        float gxv = (r0[xp] - r0[xm]) + 2.f * (r1[xp] - r1[xm]) + (r2[xp] - r2[xm]);
        float gyv = (r2[xm] - r0[xm]) + 2.f * (r2[xc] - r0[xc]) + (r2[xp] - r0[xp]);
        float vv = sqrtf(gxv * gxv + gyv * gyv);
        mag[gx + gy * g.nx] = vv;
        m = fmaxf(m, vv);
    }
    block_max_store(m, part);
}

// One separable Gaussian pass along `axis` (0 = x, 1 = y, 2 = z) (3D path).
__global__ __launch_bounds__(NTHREADS) void k_grad_blur(Geom g, const float *__restrict__ in, float *__restrict__ out,
                                                        int axis, BlurTaps taps) {
    int32_t p = blockIdx.x * NTHREADS + threadIdx.x;
    if (p >= g.n) return;
    int x, y, z;
    pixel_coords(g, p, x, y, z);
    int c = axis == 0 ? x : axis == 1 ? y : z;
    int n = axis == 0 ? g.nx : axis == 1 ? g.ny : g.nz;
    int32_t stride = axis == 0 ? 1 : axis == 1 ? g.nx : g.nx * g.ny;
    int32_t base = p - c * stride;
    float s = 0.f;
    if (c - taps.r >= 0 && c + taps.r < n) {
        const float *q = in + base + (int32_t)(c - taps.r) * stride;
        for (int k = 0; k <= 2 * taps.r; ++k) s = __fmaf_rn(taps.w[k], q[(int32_t)k * stride], s);
    } else {
        for (int k = -taps.r; k <= taps.r; ++k) {
            int j = reflect_idx(c + k, n);
            s = __fmaf_rn(taps.w[k + taps.r], in[base + j * stride], s);
        }
    }
    out[p] = s;
}

// Unnormalised Sobel magnitude (replicated borders) and its maximum.
template <int NDIM>
__global__ __launch_bounds__(NTHREADS) void k_grad_sobel(Geom g, const float *__restrict__ a, float *__restrict__ mag,
                                                         float *__restrict__ part) {
    int32_t p = blockIdx.x * NTHREADS + threadIdx.x;
    float m = 0.f;
    if (p < g.n) {
        int x, y, z;
        pixel_coords(g, p, x, y, z);
        int xm = clampi(x - 1, 0, g.nx - 1), xp = clampi(x + 1, 0, g.nx - 1);
        int ym = clampi(y - 1, 0, g.ny - 1), yp = clampi(y + 1, 0, g.ny - 1);
        const int xs[3] = {xm, x, xp};
        const int ys[3] = {ym, y, yp};
        const float w[3] = {1.f, 2.f, 1.f};
        if (NDIM == 2) {
            const float *r0 = a + (int32_t)ym * g.nx, *r1 = a + (int32_t)y * g.nx, *r2 = a + (int32_t)yp * g.nx;
            float gx = (r0[xp] - r0[xm]) + 2.f * (r1[xp] - r1[xm]) + (r2[xp] - r2[xm]);
            float gy = (r2[xm] - r0[xm]) + 2.f * (r2[x] - r0[x]) + (r2[xp] - r0[xp]);
            m = sqrtf(gx * gx + gy * gy);
        } else {
            int zm = clampi(z - 1, 0, g.nz - 1), zp = clampi(z + 1, 0, g.nz - 1);
            const int zs[3] = {zm, z, zp};
            float gx = 0.f, gy = 0.f, gz = 0.f;
            int32_t plane = g.nx * g.ny;
            for (int j = 0; j < 3; ++j)
                for (int i = 0; i < 3; ++i) {
                    // gx: derivative along x, smoothing along y (i) and z (j)
                    const float *rx = a + (int32_t)zs[j] * plane + (int32_t)ys[i] * g.nx;
                    gx += w[i] * w[j] * (rx[xp] - rx[xm]);
                    // gy: derivative along y, smoothing along x (i) and z (j)
                    const float *ry = a + (int32_t)zs[j] * plane;
                    gy += w[i] * w[j] * (ry[(int32_t)yp * g.nx + xs[i]] - ry[(int32_t)ym * g.nx + xs[i]]);
                    // gz: derivative along z, smoothing along x (i) and y (j)
                    gz += w[i] * w[j] * (a[(int32_t)zp * plane + (int32_t)ys[j] * g.nx + xs[i]] -
                                         a[(int32_t)zm * plane + (int32_t)ys[j] * g.nx + xs[i]]);
                }
            m = sqrtf(gx * gx + gy * gy + gz * gz);
        }
        mag[p] = m;
    }
    block_max_store(m, part);
}

template <typename T>
__global__ __launch_bounds__(NTHREADS) void k_grad_quant(int32_t n, const float *__restrict__ mag, T *__restrict__ out,
                                                         const float *__restrict__ gmax, float Q) {
    const float mx = *gmax;
    for (int32_t p = blockIdx.x * NTHREADS * 4 + threadIdx.x; p < n && p < (blockIdx.x + 1) * NTHREADS * 4; p += NTHREADS) {
        float v = 0.f;
        if (mx > 0.f) v = rintf(__fdiv_rn(mag[p] * Q, mx));
        v = fminf(fmaxf(v, 0.f), Q);
        out[p] = (T)v;
    }
}

int grad_parts(const Geom &g, int ndim, int r) {
    if (ndim == 2 && r <= FUSED_MAX_R) return ((g.nx + GX - 1) / GX) * ((g.ny + GY - 1) / GY);
    return (g.n + NTHREADS - 1) / NTHREADS;
}

// Taps of radius r re-centred on radius RB >= r, zero beyond r.
static BlurTaps pad_taps(const BlurTaps &taps, int RB) {
    BlurTaps p;
    p.r = RB;
    for (int k = 0; k <= 2 * RB; ++k) {
        int o = k - RB;
        p.w[k] = (o >= -taps.r && o <= taps.r) ? taps.w[o + taps.r] : 0.f;
    }
    return p;
}

int launch_grad_fused2d(Launch &lc, const Geom &g, const float *img, float *mag, float *part, const BlurTaps &taps) {
    int tiles = ((g.nx + GX - 1) / GX) * ((g.ny + GY - 1) / GY);
    if (taps.r == 0)
        return lc.run("grad_fused", k_grad_fused2d<0>, dim3(tiles), dim3(NTHREADS), g, img, mag, part, pad_taps(taps, 0));
    if (taps.r <= 4)
        return lc.run("grad_fused", k_grad_fused2d<4>, dim3(tiles), dim3(NTHREADS), g, img, mag, part, pad_taps(taps, 4));
    if (taps.r <= 8)
        return lc.run("grad_fused", k_grad_fused2d<8>, dim3(tiles), dim3(NTHREADS), g, img, mag, part, pad_taps(taps, 8));
    return lc.run("grad_fused", k_grad_fused2d<16>, dim3(tiles), dim3(NTHREADS), g, img, mag, part, pad_taps(taps, 16));
}
int launch_grad_blur(Launch &lc, const Geom &g, const float *in, float *out, int axis, const BlurTaps &taps) {
    return lc.run("grad_blur", k_grad_blur, dim3((g.n + NTHREADS - 1) / NTHREADS), dim3(NTHREADS), g, in, out, axis, taps);
}
int launch_grad_sobel(Launch &lc, const Geom &g, int ndim, const float *a, float *mag, float *part) {
    if (ndim == 3)
        return lc.run("grad_sobel", k_grad_sobel<3>, dim3((g.n + NTHREADS - 1) / NTHREADS), dim3(NTHREADS), g, a, mag, part);
    return lc.run("grad_sobel", k_grad_sobel<2>, dim3((g.n + NTHREADS - 1) / NTHREADS), dim3(NTHREADS), g, a, mag, part);
}
// Maximum of nparts partial maxima into *gmax: one workgroup per 64 Ki
// partials (at most 256), then one more for their maxima; tmp holds 256 floats.
int launch_grad_max(Launch &lc, int32_t nparts, const float *part, float *tmp, float *gmax) {
    int32_t G = (nparts + 65535) / 65536;
    if (G <= 1) return lc.run("grad_max", k_grad_max, dim3(1), dim3(NTHREADS), nparts, part, gmax);
    if (G > 256) G = 256;
    int rc = lc.run("grad_max", k_grad_max, dim3(G), dim3(NTHREADS), nparts, part, tmp);
    if (rc) return rc;
    return lc.run("grad_max", k_grad_max, dim3(1), dim3(NTHREADS), G, (const float *)tmp, gmax);
}
int launch_grad_quant(Launch &lc, int32_t n, bool u16, const float *mag, void *out, const float *gmax) {
    dim3 grid((n + NTHREADS * 4 - 1) / (NTHREADS * 4));
    if (u16)
        return lc.run("grad_quant", k_grad_quant<uint16_t>, grid, dim3(NTHREADS), n, mag, (uint16_t *)out, gmax, 65535.f);
    return lc.run("grad_quant", k_grad_quant<uint8_t>, grid, dim3(NTHREADS), n, mag, (uint8_t *)out, gmax, 255.f);
}

}  // namespace wsk
