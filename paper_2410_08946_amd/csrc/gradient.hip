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
// use separable passes. The global maximum is kept in MAXSLOTS words (one per
// group of workgroups) to spread the atomics; the quantiser reduces the slots.
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

// Block maximum of non-negative floats, one atomic into slot blockIdx % MAXSLOTS
// (non-negative floats order like their bit patterns).
__device__ __forceinline__ void block_max_to_slot(float m, unsigned int *slots) {
    __shared__ float wmax[NTHREADS / 64];
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    if (__lane_id() == 0) wmax[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        float b = wmax[0];
        for (int w = 1; w < NTHREADS / 64; ++w) b = fmaxf(b, wmax[w]);
        atomicMax(slots + (blockIdx.x % MAXSLOTS), __float_as_uint(b));
    }
}

// ---------------------------------------------------------------------------
// Fused 2D gradient: tile of GX x GY magnitudes per workgroup.
// LDS: raw (GY+2+2r) x (GX+2+2r), x-blurred (GY+2+2r) x (GX+2), blurred
// (GY+2) x (GX+2); virtual coordinates outside the image are mirrored for the
// blur; the Sobel stencil clamps to the image (replicated border).
// ---------------------------------------------------------------------------
constexpr int GX = 64, GY = 16;

// RB bounds the blur radius of the instantiation (the loads of the raw tile
// are unrolled for it); the taps' runtime radius r <= RB sizes the LDS tile.
template <int RB>
__global__ __launch_bounds__(NTHREADS) void k_grad_fused2d(Geom g, const float *__restrict__ img,
                                                           float *__restrict__ mag, unsigned int *__restrict__ slots,
                                                           BlurTaps taps) {
    extern __shared__ float smem[];
    const int r = taps.r;
    const int RW = GX + 2 + 2 * r, RH = GY + 2 + 2 * r;  // raw
    const int BW = GX + 2;                               // blurred widths
    float *raw = smem;
    float *bx = raw + RW * RH;
    float *bb = bx + BW * RH;
    int tiles_x = (g.nx + GX - 1) / GX;
    int x0 = (blockIdx.x % tiles_x) * GX, y0 = (blockIdx.x / tiles_x) * GY;
    {
        // batched raw loads: mirrored addresses first, then all loads
        constexpr int PER = ((GX + 2 + 2 * RB) * (GY + 2 + 2 * RB) + NTHREADS - 1) / NTHREADS;
        int32_t idx[PER];
        float v[PER];
        const int cells = RW * RH;
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            int c = threadIdx.x + j * NTHREADS;
            int i = c % RW, jj = c / RW;
            int gx = reflect_idx(x0 - 1 - r + i, g.nx), gy = reflect_idx(y0 - 1 - r + jj, g.ny);
            idx[j] = c < cells ? gx + (int32_t)gy * g.nx : 0;
        }
#pragma unroll
        for (int j = 0; j < PER; ++j) v[j] = img[idx[j]];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            int c = threadIdx.x + j * NTHREADS;
            if (c < cells) raw[c] = v[j];
        }
    }
    __syncthreads();
    for (int c = threadIdx.x; c < BW * RH; c += NTHREADS) {
        int i = c % BW, j = c / BW;
        const float *row = raw + j * RW + i;  // virtual x = x0-1+i-r+k at row[k]
        float s = 0.f;
        for (int k = 0; k <= 2 * r; ++k) s = __fmaf_rn(taps.w[k], row[k], s);
        bx[c] = s;
    }
    __syncthreads();
    for (int c = threadIdx.x; c < BW * (GY + 2); c += NTHREADS) {
        int i = c % BW, j = c / BW;
        const float *col = bx + j * BW + i;
        float s = 0.f;
        for (int k = 0; k <= 2 * r; ++k) s = __fmaf_rn(taps.w[k], col[k * BW], s);
        bb[c] = s;
    }
    __syncthreads();
    float m = 0.f;
    for (int c = threadIdx.x; c < GX * GY; c += NTHREADS) {
        int i = c % GX, j = c / GX;
        int gx = x0 + i, gy = y0 + j;
        if (gx >= g.nx || gy >= g.ny) continue;
        // local columns/rows of the clamped neighbours (+1 for the ring)
        int xm = clampi(gx - 1, 0, g.nx - 1) - x0 + 1, xp = clampi(gx + 1, 0, g.nx - 1) - x0 + 1, xc = i + 1;
        int ym = clampi(gy - 1, 0, g.ny - 1) - y0 + 1, yp = clampi(gy + 1, 0, g.ny - 1) - y0 + 1, yc = j + 1;
        const float *r0 = bb + ym * BW, *r1 = bb + yc * BW, *r2 = bb + yp * BW;
        float gxv = (r0[xp] - r0[xm]) + 2.f * (r1[xp] - r1[xm]) + (r2[xp] - r2[xm]);
        float gyv = (r2[xm] - r0[xm]) + 2.f * (r2[xc] - r0[xc]) + (r2[xp] - r0[xp]);
        float vv = sqrtf(gxv * gxv + gyv * gyv);
        mag[gx + (int32_t)gy * g.nx] = vv;
        m = fmaxf(m, vv);
    }
    block_max_to_slot(m, slots);
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
                                                         unsigned int *__restrict__ slots) {
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
    block_max_to_slot(m, slots);
}

template <typename T>
__global__ __launch_bounds__(NTHREADS) void k_grad_quant(int32_t n, const float *__restrict__ mag, T *__restrict__ out,
                                                         const unsigned int *__restrict__ slots, float Q) {
    __shared__ float smax;
    if (threadIdx.x < 64) {
        float m = 0.f;
        for (int s = threadIdx.x; s < MAXSLOTS; s += 64) m = fmaxf(m, __uint_as_float(slots[s]));
        for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
        if (threadIdx.x == 0) smax = m;
    }
    __syncthreads();
    float mx = smax;
    for (int32_t p = blockIdx.x * NTHREADS * 4 + threadIdx.x; p < n && p < (blockIdx.x + 1) * NTHREADS * 4; p += NTHREADS) {
        float v = 0.f;
        if (mx > 0.f) v = rintf(__fdiv_rn(mag[p] * Q, mx));
        v = fminf(fmaxf(v, 0.f), Q);
        out[p] = (T)v;
    }
}

__global__ void k_grad_zero_slots(unsigned int *slots) {
    for (int i = threadIdx.x; i < MAXSLOTS; i += blockDim.x) slots[i] = 0u;
}

size_t grad_fused2d_lds(int r) {
    int RW = GX + 2 + 2 * r, RH = GY + 2 + 2 * r, BW = GX + 2;
    return sizeof(float) * (size_t)(RW * RH + BW * RH + BW * (GY + 2));
}

int launch_grad_fused2d(Launch &lc, const Geom &g, const float *img, float *mag, unsigned int *slots, const BlurTaps &taps) {
    int tiles = ((g.nx + GX - 1) / GX) * ((g.ny + GY - 1) / GY);
    size_t shm = grad_fused2d_lds(taps.r);
    if (taps.r == 0)
        return lc.run_shm("grad_fused", k_grad_fused2d<0>, dim3(tiles), dim3(NTHREADS), shm, g, img, mag, slots, taps);
    if (taps.r <= 4)
        return lc.run_shm("grad_fused", k_grad_fused2d<4>, dim3(tiles), dim3(NTHREADS), shm, g, img, mag, slots, taps);
    if (taps.r <= 8)
        return lc.run_shm("grad_fused", k_grad_fused2d<8>, dim3(tiles), dim3(NTHREADS), shm, g, img, mag, slots, taps);
    return lc.run_shm("grad_fused", k_grad_fused2d<16>, dim3(tiles), dim3(NTHREADS), shm, g, img, mag, slots, taps);
}
int launch_grad_blur(Launch &lc, const Geom &g, const float *in, float *out, int axis, const BlurTaps &taps) {
    return lc.run("grad_blur", k_grad_blur, dim3((g.n + NTHREADS - 1) / NTHREADS), dim3(NTHREADS), g, in, out, axis, taps);
}
int launch_grad_sobel(Launch &lc, const Geom &g, int ndim, const float *a, float *mag, unsigned int *slots) {
    if (ndim == 3)
        return lc.run("grad_sobel", k_grad_sobel<3>, dim3((g.n + NTHREADS - 1) / NTHREADS), dim3(NTHREADS), g, a, mag, slots);
    return lc.run("grad_sobel", k_grad_sobel<2>, dim3((g.n + NTHREADS - 1) / NTHREADS), dim3(NTHREADS), g, a, mag, slots);
}
int launch_grad_quant(Launch &lc, int32_t n, bool u16, const float *mag, void *out, const unsigned int *slots) {
    dim3 grid((n + NTHREADS * 4 - 1) / (NTHREADS * 4));
    if (u16)
        return lc.run("grad_quant", k_grad_quant<uint16_t>, grid, dim3(NTHREADS), n, mag, (uint16_t *)out, slots, 65535.f);
    return lc.run("grad_quant", k_grad_quant<uint8_t>, grid, dim3(NTHREADS), n, mag, (uint8_t *)out, slots, 255.f);
}
int launch_grad_zero_slots(Launch &lc, unsigned int *slots) {
    return lc.run("grad_zero", k_grad_zero_slots, dim3(1), dim3(64), slots);
}

}  // namespace wsk
