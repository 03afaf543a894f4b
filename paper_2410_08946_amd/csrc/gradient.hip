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
// use separable blur passes and a z-marching Sobel kernel. Every workgroup stores its maximum in its own word (no
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
    // rows padded to whole float4s: the blurs compute 4 outputs per item from
    // 16-byte LDS reads (the 2 extra columns per row are never read back)
    constexpr int BQ = (BW + 3) / 4;          // float4 blocks per blurred row
    constexpr int BWP = 4 * BQ;               // blurred row pitch
    constexpr int RWP = BWP + 2 * RB + ((BWP + 2 * RB) % 4 ? 4 - (BWP + 2 * RB) % 4 : 0);  // raw row pitch
    static_assert(RWP >= RW && RWP % 4 == 0, "raw pitch");
    __shared__ __align__(16) float raw[RWP * RH];
    __shared__ __align__(16) float bx[BWP * RH];
    __shared__ __align__(16) float bb[BWP * BH];
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
            if (c < CELLS) raw[(c / RW) * RWP + c % RW] = v[j];
        }
    }
    __syncthreads();
    // x blur: item = (row, block of 4 columns); output column i reads raw
    // columns i .. i + 2RB of its row (the taps in order, as before)
    for (int c = threadIdx.x; c < BQ * RH; c += NTHREADS) {
        const int r = c / BQ, q = c % BQ;
        const float4 *row = (const float4 *)(raw + r * RWP + 4 * q);
        float in[4 + 2 * RB + 3];
#pragma unroll
        for (int u = 0; u < (4 + 2 * RB + 3) / 4; ++u) {
            float4 f = row[u];
            in[4 * u] = f.x;
            in[4 * u + 1] = f.y;
            in[4 * u + 2] = f.z;
            in[4 * u + 3] = f.w;
        }
        float o[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            float s = 0.f;
#pragma unroll
            for (int k = 0; k < NT; ++k) s = __fmaf_rn(w[k], in[e + k], s);
            o[e] = s;
        }
        *(float4 *)(bx + r * BWP + 4 * q) = make_float4(o[0], o[1], o[2], o[3]);
    }
    __syncthreads();
    // y blur: item = (row, block of 4 columns); rows j .. j+2RB in order
    for (int c = threadIdx.x; c < BQ * BH; c += NTHREADS) {
        const int j = c / BQ, q = c % BQ;
        float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int k = 0; k < NT; ++k) {
            float4 f = *(const float4 *)(bx + (j + k) * BWP + 4 * q);
            s.x = __fmaf_rn(w[k], f.x, s.x);
            s.y = __fmaf_rn(w[k], f.y, s.y);
            s.z = __fmaf_rn(w[k], f.z, s.z);
            s.w = __fmaf_rn(w[k], f.w, s.w);
        }
        *(float4 *)(bb + j * BWP + 4 * q) = s;
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
        const float *r0 = bb + ym * BWP, *r1 = bb + yc * BWP, *r2 = bb + yp * BWP;
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

// Unnormalised Sobel magnitude (replicated borders) and its maximum, one
// thread per pixel (2D images whose blur radius exceeds the fused kernel's).
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

// 3D Sobel magnitude, separable and marching along z. A workgroup owns an
// S3X x S3Y column of a slab of S3Z planes; every plane it touches (the slab
// and one plane on each side) is staged with a one-voxel halo in LDS, using
// clamped coordinates (replicated border). From a plane's 3 x 3 neighbourhood
// a thread forms the plane partials
//   A = [1 2 1]_y [-1 0 1]_x a,  B = [1 2 1]_y [1 2 1]_x a,  C = [-1 0 1]_y [1 2 1]_x a,
// and from three consecutive planes
//   gx = A(z-1) + 2 A(z) + A(z+1),  gy = C(z-1) + 2 C(z) + C(z+1),  gz = B(z+1) - B(z-1),
// the unnormalised Sobel derivatives. Each voxel is read from HBM about once
// (plus halos) instead of 54 times through the cache hierarchy.
constexpr int S3X = 32, S3Y = 8, S3Z = 32;
constexpr int S3W = S3X + 2, S3H = S3Y + 2, S3CELLS = S3W * S3H;
static_assert(S3X * S3Y == NTHREADS, "one column per thread");
static_assert(S3CELLS <= 2 * NTHREADS, "two staging loads per thread");

__global__ __launch_bounds__(NTHREADS) void k_grad_sobel3(Geom g, int32_t nblocks, const float *__restrict__ a,
                                                          float *__restrict__ mag, float *__restrict__ part) {
    __shared__ float sp[2][S3CELLS];
    if ((int32_t)blockIdx.x >= nblocks) return;
    const int b = xcd_tile(blockIdx.x, nblocks);
    const int ntx = (g.nx + S3X - 1) / S3X, nty = (g.ny + S3Y - 1) / S3Y;
    const int x0 = (b % ntx) * S3X, y0 = ((b / ntx) % nty) * S3Y, zlo = (b / ntx / nty) * S3Z;
    const int tx = threadIdx.x % S3X, ty = threadIdx.x / S3X;
    const int x = x0 + tx, y = y0 + ty;
    const bool own = x < g.nx && y < g.ny;
    const int32_t plane = g.nx * g.ny;
    // staging cells of this thread (clamped source offsets within a plane)
    int32_t src[2];
    bool has[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        int c = threadIdx.x + h * NTHREADS;
        has[h] = c < S3CELLS;
        int cy = c / S3W, cx = c % S3W;
        src[h] = (int32_t)clampi(y0 - 1 + cy, 0, g.ny - 1) * g.nx + clampi(x0 - 1 + cx, 0, g.nx - 1);
    }
    const int jmax = min(S3Z + 1, g.nz - zlo + 1);  // planes zlo-1 .. zlo+jmax-1 (clamped)
    float A0 = 0.f, A1 = 0.f, B0 = 0.f, B1 = 0.f, C0 = 0.f, C1 = 0.f, m = 0.f;
    // the staging values of plane j + 1 are loaded into registers before
    // plane j is computed, so their latency overlaps the computation
    float nv[2];
    auto load_plane = [&](int j) {
        const float *pa = a + (size_t)clampi(zlo - 1 + j, 0, g.nz - 1) * (size_t)plane;
#pragma unroll
        for (int h = 0; h < 2; ++h) nv[h] = has[h] ? pa[src[h]] : 0.f;
    };
    load_plane(0);
    for (int j = 0; j <= jmax; ++j) {
        float *cur = sp[j & 1];
#pragma unroll
        for (int h = 0; h < 2; ++h)
            if (has[h]) cur[threadIdx.x + h * NTHREADS] = nv[h];
        __syncthreads();
        if (j < jmax) load_plane(j + 1);
        const float *r0 = cur + ty * S3W + tx, *r1 = r0 + S3W, *r2 = r1 + S3W;
        float d0 = r0[2] - r0[0], d1 = r1[2] - r1[0], d2 = r2[2] - r2[0];
        float s0 = r0[0] + 2.f * r0[1] + r0[2], s1 = r1[0] + 2.f * r1[1] + r1[2], s2 = r2[0] + 2.f * r2[1] + r2[2];
        float A2 = d0 + 2.f * d1 + d2, B2 = s0 + 2.f * s1 + s2, C2 = s2 - s0;
        if (j >= 2) {
            const int zo = zlo + j - 2;
            float gx = A0 + 2.f * A1 + A2, gy = C0 + 2.f * C1 + C2, gz = B2 - B0;
            float v = sqrtf(gx * gx + gy * gy + gz * gz);
            if (own) {
                mag[(size_t)zo * (size_t)plane + (size_t)y * g.nx + x] = v;
                m = fmaxf(m, v);
            }
        }
        A0 = A1;
        A1 = A2;
        B0 = B1;
        B1 = B2;
        C0 = C1;
        C1 = C2;
        // the next plane goes to the other buffer; the barrier after its
        // staging orders this plane's reads before that buffer's reuse
    }
    block_max_store(m, part);
}

// g_q = rint(mag Q / max) clamped to [0, Q], 0 when the maximum is 0. A
// thread quantises 4 consecutive pixels: one 16-byte load when vec & 2 (the
// magnitudes are 16-byte aligned) and one 4- or 8-byte store when vec & 1 (the
// output is aligned for it).
template <typename T> struct Vec4;
template <> struct Vec4<uint8_t> { using type = uchar4; };
template <> struct Vec4<uint16_t> { using type = ushort4; };

template <typename T>
__global__ __launch_bounds__(NTHREADS) void k_grad_quant(int32_t n, const float *__restrict__ mag, T *__restrict__ out,
                                                         const float *__restrict__ gmax, float Q, int vec) {
    const float mx = *gmax;
    const int32_t p = (int32_t)(blockIdx.x * NTHREADS + threadIdx.x) * 4;
    if (p >= n) return;
    const bool full = p + 3 < n;
    float v[4];
    if (full && (vec & 2)) {
        float4 q = *(const float4 *)(mag + p);
        v[0] = q.x;
        v[1] = q.y;
        v[2] = q.z;
        v[3] = q.w;
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = p + e < n ? mag[p + e] : 0.f;
    }
    T o[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        float u = 0.f;
        if (mx > 0.f) u = rintf(__fdiv_rn(v[e] * Q, mx));
        o[e] = (T)fminf(fmaxf(u, 0.f), Q);
    }
    if (full && (vec & 1)) {
        typename Vec4<T>::type w;
        w.x = o[0];
        w.y = o[1];
        w.z = o[2];
        w.w = o[3];
        *(typename Vec4<T>::type *)(out + p) = w;
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (p + e < n) out[p + e] = o[e];
    }
}

static int32_t sobel3_blocks(const Geom &g) {
    return ((g.nx + S3X - 1) / S3X) * ((g.ny + S3Y - 1) / S3Y) * ((g.nz + S3Z - 1) / S3Z);
}

int grad_parts(const Geom &g, int ndim, int r) {
    if (ndim == 2 && r <= FUSED_MAX_R) return ((g.nx + GX - 1) / GX) * ((g.ny + GY - 1) / GY);
    if (ndim == 3) return sobel3_blocks(g);
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
    if (ndim == 3) {
        int32_t nb = sobel3_blocks(g);
        return lc.run("grad_sobel", k_grad_sobel3, dim3(nb), dim3(NTHREADS), g, nb, a, mag, part);
    }
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
    dim3 grid((uint32_t)(((int64_t)n + NTHREADS * 4 - 1) / (NTHREADS * 4)));
    const int vec = (((uintptr_t)out % (u16 ? 8 : 4)) == 0 ? 1 : 0) | (((uintptr_t)mag % 16) == 0 ? 2 : 0);
    if (u16)
        return lc.run("grad_quant", k_grad_quant<uint16_t>, grid, dim3(NTHREADS), n, mag, (uint16_t *)out, gmax, 65535.f,
                      vec);
    return lc.run("grad_quant", k_grad_quant<uint8_t>, grid, dim3(NTHREADS), n, mag, (uint8_t *)out, gmax, 255.f, vec);
}

}  // namespace wsk
