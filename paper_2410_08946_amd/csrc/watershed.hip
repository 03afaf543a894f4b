// watershed.hip -- generic parts of the watershed transform (Alg. 1) on
// gfx950: the step-level output kernel, fills, and the launchers that pick
// the tile kernels of a tile shape (ws_tiles.h; each shape's kernels are
// compiled in ws_shape.hip).
//
// Step II is computed as the unique fixpoint of
//   D(p) = 1 + min{ D(q) : q in N(p), I(q) = I(p) }      (plateau pixels)
// (see ws_tiles.h for the data on the device and the tile schedule).
#include "ws_tiles.h"

namespace wsk {

// ---------------------------------------------------------------------------
// Arrow of one pixel from global memory (same rules as lds_arrow), used by
// the step-level output kernel. Returns the target pixel, -1 for a root, -2
// for a minimal plateau pixel.
// ---------------------------------------------------------------------------
template <int CONN, typename T>
__device__ __forceinline__ int32_t glb_arrow(const Geom &g, const T *__restrict__ I, const int32_t *__restrict__ D,
                                             int x, int y, int z, int32_t p, int32_t *state_out, int32_t *eq1_out) {
    int32_t r[CONN];
    bool ok[CONN];
#pragma unroll
    for (int k = 0; k < CONN; ++k) {
        int xx = x + nb_dx<CONN>(k), yy = y + nb_dy<CONN>(k), zz = z + nb_dz<CONN>(k);
        ok[k] = in_image(g, xx, yy, zz);
        r[k] = ok[k] ? xx + g.nx * (yy + g.ny * zz) : p;
    }
    int w[CONN], dq[CONN];
#pragma unroll
    for (int k = 0; k < CONN; ++k) w[k] = I[r[k]];
#pragma unroll
    for (int k = 0; k < CONN; ++k) dq[k] = D[r[k]];
    int v = I[p], d = D[p];
    int m = SENT;
    int32_t q = p;
#pragma unroll
    for (int k = 0; k < CONN; ++k)
        if (ok[k] && w[k] <= m) { m = w[k]; q = r[k]; }
    int state = (m > v) ? 1 : (m < v) ? 0 : (q > p ? 2 : 3);
    *state_out = state;
    *eq1_out = q;
    if (d == INF) return -2;
    if (d == 0) return state == 0 ? q : -1;
#pragma unroll
    for (int k = 0; k < CONN; ++k)
        if (ok[k] && w[k] == v && dq[k] == d - 1) return r[k];
    return -1;
}

// Step-level outputs (balanced state encoding and arrows) for verification.
template <int CONN, typename T>
__global__ __launch_bounds__(NTHREADS) void k_ws_stages(Geom g, const T *__restrict__ I, const int32_t *__restrict__ D,
                                                        int32_t *__restrict__ bal, int32_t *__restrict__ arrow) {
    int32_t p = blockIdx.x * NTHREADS + threadIdx.x;
    if (p >= g.n) return;
    int x, y, z;
    pixel_coords(g, p, x, y, z);
    int state = 1;
    int32_t eq1 = p;
    int32_t q = glb_arrow<CONN, T>(g, I, D, x, y, z, p, &state, &eq1);
    int d = D[p];
    if (d != 0 && d != INF) {
        bal[p] = -d;
        arrow[p] = q;
        return;
    }
    bal[p] = state;
    arrow[p] = (state == 0 || state == 2) ? eq1 : p;  // Eq. (1) target, or a self loop
}

__global__ void k_fill_i32(int32_t *a, int32_t n, int32_t v) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

// Two fills in one launch: a[0, na) = va, then b[0, nb) = vb.
__global__ void k_fill2_i32(int32_t *a, int32_t na, int32_t va, int32_t *b, int32_t nb, int32_t vb) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < na) a[i] = va;
    else if (i - na < nb) b[i - na] = vb;
}

// ---------------------------------------------------------------------------
// Host-side launchers.
// ---------------------------------------------------------------------------
template <int CONN, typename T>
static int launch_ws_stages_t(Launch &lc, const Geom &g, const void *I, const int32_t *D, int32_t *bal, int32_t *arrow) {
    return lc.run("ws_stages", k_ws_stages<CONN, T>, dim3((g.n + NTHREADS - 1) / NTHREADS), dim3(NTHREADS), g,
                  (const T *)I, D, bal, arrow);
}

#define WS_DISPATCH(FN, conn, u16, ...)                                                  \
    switch (conn) {                                                                      \
    case 4: return u16 ? FN<4, uint16_t>(__VA_ARGS__) : FN<4, uint8_t>(__VA_ARGS__);     \
    case 8: return u16 ? FN<8, uint16_t>(__VA_ARGS__) : FN<8, uint8_t>(__VA_ARGS__);     \
    case 6: return u16 ? FN<6, uint16_t>(__VA_ARGS__) : FN<6, uint8_t>(__VA_ARGS__);     \
    case 26: return u16 ? FN<26, uint16_t>(__VA_ARGS__) : FN<26, uint8_t>(__VA_ARGS__);  \
    default: return -1;                                                                  \
    }

// The launcher `FN` of the shape's WsShape.
#define WS_BY_SHAPE(FN, shape, ...)                         \
    switch (shape) {                                        \
    case 2: return WsShape<2>::FN(__VA_ARGS__);             \
    case 12: return WsShape<12>::FN(__VA_ARGS__);           \
    case 22: return WsShape<22>::FN(__VA_ARGS__);           \
    case 32: return WsShape<32>::FN(__VA_ARGS__);           \
    case 3: return WsShape<3>::FN(__VA_ARGS__);             \
    case 13: return WsShape<13>::FN(__VA_ARGS__);           \
    case 23: return WsShape<23>::FN(__VA_ARGS__);           \
    case 33: return WsShape<33>::FN(__VA_ARGS__);           \
    default: return -1;                                     \
    }

#define WS_SRC_FUNCS(Src)                                                                                          \
    int launch_ws_init(Launch &lc, const Src &src, const TileGrid &tg, int conn, int shape, bool u16, int32_t *D, \
                       int32_t *stamp, int32_t *changed) {                                                         \
        WS_BY_SHAPE(init, shape, lc, src, tg, conn, u16, D, stamp, changed)                                        \
    }                                                                                                              \
    int launch_ws_sweep(Launch &lc, const Src &src, const TileGrid &tg, int conn, int shape, bool u16,            \
                        int32_t *D, int32_t *stamp, int32_t *changed, const int32_t *prev, int32_t s) {            \
        WS_BY_SHAPE(sweep, shape, lc, src, tg, conn, u16, D, stamp, changed, prev, s)                              \
    }                                                                                                              \
    int launch_ws_label(Launch &lc, const Src &src, const TileGrid &tg, int conn, int shape, bool u16,            \
                        const int32_t *D, int32_t *rec) {                                                          \
        WS_BY_SHAPE(label, shape, lc, src, tg, conn, u16, D, rec)                                                  \
    }                                                                                                              \
    int launch_ws_merge(Launch &lc, const Src &src, const TileGrid &tg, int conn, int shape, bool u16,            \
                        const int32_t *rec) {                                                                      \
        WS_BY_SHAPE(merge, shape, lc, src, tg, conn, u16, rec)                                                     \
    }                                                                                                              \
    int launch_ws_find(Launch &lc, const Src &src, const TileGrid &tg, int conn, int shape) {                     \
        WS_BY_SHAPE(find, shape, lc, src, tg, conn)                                                                \
    }                                                                                                              \
    int launch_ws_jump(Launch &lc, const Src &src, const TileGrid &tg, int conn, int shape, int32_t rr,           \
                       int32_t *changed) {                                                                         \
        WS_BY_SHAPE(jump, shape, lc, src, tg, conn, rr, changed)                                                   \
    }

WS_SRC_FUNCS(OneImg)
WS_SRC_FUNCS(ImgTable)

int launch_ws_stages(Launch &lc, const Geom &g, int conn, bool u16, const void *I, const int32_t *D, int32_t *bal,
                     int32_t *arrow) {
    WS_DISPATCH(launch_ws_stages_t, conn, u16, lc, g, I, D, bal, arrow)
}
int launch_fill_i32(Launch &lc, int32_t *a, int32_t n, int32_t v) {
    if (n <= 0) return 0;
    return lc.run("fill", k_fill_i32, dim3((n + 255) / 256), dim3(256), a, n, v);
}
int launch_fill2_i32(Launch &lc, int32_t *a, int32_t na, int32_t va, int32_t *b, int32_t nb, int32_t vb) {
    const int64_t n = (int64_t)na + nb;
    if (n <= 0) return 0;
    return lc.run("fill", k_fill2_i32, dim3((uint32_t)((n + 255) / 256)), dim3(256), a, na, va, b, nb, vb);
}
int record_ints(int shape) {
    switch (shape) {
    case 2: return Border<2>::RS;
    case 12: return Border<12>::RS;
    case 22: return Border<22>::RS;
    case 32: return Border<32>::RS;
    case 3: return Border<3>::RS;
    case 13: return Border<13>::RS;
    case 23: return Border<23>::RS;
    case 33: return Border<33>::RS;
    default: return 0;
    }
}

}  // namespace wsk
