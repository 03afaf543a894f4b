// gradient.hip -- gfx950 kernels of the gradient pre-processing (Introduction:
// smooth the image minimally, then take the gradient magnitude; both optional
// before Step I per the PRUF pipeline figure).
//
// float32 throughout. Per pixel the summation order is fixed (taps from -r to
// +r; Sobel terms in a fixed order), so the result does not depend on the
// launch configuration or on which other images are processed alongside.
#include "ws_device.h"
#include "ws_kernels.h"

namespace wsk {

__device__ __forceinline__ int reflect_idx(int i, int n) {
    // half-sample symmetric borders: ... c b a | a b c ... (period 2n)
    int m = 2 * n;
    i %= m;
    if (i < 0) i += m;
    return i < n ? i : m - 1 - i;
}

// One separable Gaussian pass along `axis` (0 = x, 1 = y, 2 = z).
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
    for (int k = -taps.r; k <= taps.r; ++k) {
        int j = reflect_idx(c + k, n);
        s = __fmaf_rn(taps.w[k + taps.r], in[base + j * stride], s);
    }
    out[p] = s;
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Unnormalised Sobel magnitude (replicated borders) and its maximum.
template <int NDIM>
__global__ __launch_bounds__(NTHREADS) void k_grad_sobel(Geom g, const float *__restrict__ a, float *__restrict__ mag,
                                                         unsigned int *__restrict__ maxbits) {
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
    // wave maximum, then one atomic per wave (non-negative floats order like
    // their bit patterns)
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    if (__lane_id() == 0) atomicMax(maxbits, __float_as_uint(m));
}

template <typename T>
__global__ __launch_bounds__(NTHREADS) void k_grad_quant(int32_t n, const float *__restrict__ mag, T *__restrict__ out,
                                                         const unsigned int *__restrict__ maxbits, float Q) {
    int32_t p = blockIdx.x * NTHREADS + threadIdx.x;
    if (p >= n) return;
    float mx = __uint_as_float(*maxbits);
    float v = 0.f;
    if (mx > 0.f) v = rintf(__fdiv_rn(mag[p] * Q, mx));
    v = fminf(fmaxf(v, 0.f), Q);
    out[p] = (T)v;
}

__global__ void k_grad_zero_max(unsigned int *maxbits) { *maxbits = 0u; }

int launch_grad_blur(Launch &lc, const Geom &g, const float *in, float *out, int axis, const BlurTaps &taps) {
    return lc.run("grad_blur", k_grad_blur, dim3((g.n + NTHREADS - 1) / NTHREADS), dim3(NTHREADS), g, in, out, axis, taps);
}
int launch_grad_sobel(Launch &lc, const Geom &g, int ndim, const float *a, float *mag, unsigned int *maxbits) {
    if (ndim == 3)
        return lc.run("grad_sobel", k_grad_sobel<3>, dim3((g.n + NTHREADS - 1) / NTHREADS), dim3(NTHREADS), g, a, mag, maxbits);
    return lc.run("grad_sobel", k_grad_sobel<2>, dim3((g.n + NTHREADS - 1) / NTHREADS), dim3(NTHREADS), g, a, mag, maxbits);
}
int launch_grad_quant(Launch &lc, int32_t n, bool u16, const float *mag, void *out, const unsigned int *maxbits) {
    if (u16)
        return lc.run("grad_quant", k_grad_quant<uint16_t>, dim3((n + NTHREADS - 1) / NTHREADS), dim3(NTHREADS), n, mag,
                      (uint16_t *)out, maxbits, 65535.f);
    return lc.run("grad_quant", k_grad_quant<uint8_t>, dim3((n + NTHREADS - 1) / NTHREADS), dim3(NTHREADS), n, mag,
                  (uint8_t *)out, maxbits, 255.f);
}
int launch_grad_zero_max(Launch &lc, unsigned int *maxbits) {
    return lc.run("grad_zero", k_grad_zero_max, dim3(1), dim3(1), maxbits);
}

}  // namespace wsk
