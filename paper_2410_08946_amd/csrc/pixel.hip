// pixel.hip -- the per-pixel synchronous schedule of Alg. 1 (the PRUF_sync
// implementation of Section 3.3 and its PRW / APRUF variants, Sections 3.1-3.2):
// one thread per pixel, one launch per step or sweep, every decision of a sweep
// taken from the values published by the previous launch. It computes the same
// labels as the tile schedule and exists so the two designs can be compared on
// the same device.
//
// State array S (int32 per pixel) after Step I and during Step II:
//   0          a strictly lower neighbour exists (Step I state 0);
//   d >= 1     non-minimal plateau pixel resolved by sweep d (its geodesic
//              distance to the plateau's lower border);
//   PX_ST1     strict local minimum (state 1);
//   PX_ST2/3   plateau pixel not (yet) resolved, with / without an equal
//              neighbour after it (states 2 and 3); still set after Step II
//              exactly for the pixels of minimal plateaux.
// A sweep s resolves an unresolved pixel whose equal neighbour was resolved
// before the sweep (S < s), which is the synchronous state update of Step II
// with the S' buffer folded into the sweep number: writes of sweep s (value s)
// never satisfy S < s, so no pixel sees a decision of its own sweep.

#include "ws_device.h"
#include "ws_kernels.h"

namespace wsk {

constexpr int32_t PX_ST1 = 0x7ffffff1;
constexpr int32_t PX_ST2 = 0x7ffffff2;
constexpr int32_t PX_ST3 = 0x7ffffff3;
constexpr int PX_T = 256;          // threads per workgroup
constexpr int PX_SPIN = 4096;      // bound on one thread's Step IV exchange loop

__device__ __forceinline__ bool px_index(const Geom &g, int32_t &p) {
    uint32_t u = blockIdx.x * (uint32_t)PX_T + threadIdx.x;
    p = (int32_t)u;
    return u < (uint32_t)g.n;
}

// One count per wave of the lanes with `pred` set.
__device__ __forceinline__ void px_count(bool pred, int32_t *counter) {
    uint64_t m = __ballot(pred);
    if (m != 0 && __lane_id() == __ffsll((unsigned long long)m) - 1) atomicAdd(counter, __popcll(m));
}

// Neighbour k of p at (x, y, z), or -1 outside the image.
template <int CONN>
__device__ __forceinline__ int32_t px_nb(const Geom &g, int32_t p, int x, int y, int z, int k) {
    int dx = nb_dx<CONN>(k), dy = nb_dy<CONN>(k), dz = nb_dz<CONN>(k);
    if (!in_image(g, x + dx, y + dy, z + dz)) return -1;
    return p + dx + g.nx * (dy + g.ny * dz);
}

template <int CONN> __host__ __device__ constexpr int px_nnb() { return CONN == 26 ? 26 : CONN; }

// Step I (Eq. (1)): q = the last of the lowest neighbours in pixel order.
template <int CONN, typename T>
__global__ __launch_bounds__(PX_T) void k_px_step1(Geom g, const T *__restrict__ I, int32_t *__restrict__ L,
                                                   int32_t *__restrict__ S) {
    int32_t p;
    if (!px_index(g, p)) return;
    int x, y, z;
    pixel_coords(g, p, x, y, z);
    const int32_t ip = I[p];
    int32_t m = 0x7fffffff, q = -1;
#pragma unroll
    for (int k = 0; k < px_nnb<CONN>(); ++k) {
        int32_t r = px_nb<CONN>(g, p, x, y, z, k);
        if (r < 0) continue;
        int32_t v = I[r];
        if (v <= m) {
            m = v;
            q = r;
        }
    }
    int32_t st, l = p;
    if (q < 0 || m > ip) {
        st = PX_ST1;
    } else if (m < ip) {
        st = 0;
        l = q;
    } else if (q > p) {
        st = PX_ST2;
        l = q;
    } else {
        st = PX_ST3;
    }
    L[p] = l;
    S[p] = st;
}

// Step II, sweep s: an unresolved plateau pixel with an equal neighbour that was
// resolved before this sweep points to the first such neighbour in pixel order.
template <int CONN, typename T>
__global__ __launch_bounds__(PX_T) void k_px_sweep(Geom g, const T *__restrict__ I, int32_t *__restrict__ L,
                                                   int32_t *__restrict__ S, int32_t s, int32_t *__restrict__ changed) {
    int32_t p;
    bool hit = false;
    if (px_index(g, p) && S[p] >= PX_ST2) {
        int x, y, z;
        pixel_coords(g, p, x, y, z);
        const int32_t ip = I[p];
        for (int k = 0; k < px_nnb<CONN>(); ++k) {
            int32_t r = px_nb<CONN>(g, p, x, y, z, k);
            if (r < 0 || (int32_t)I[r] != ip || S[r] >= s) continue;
            S[p] = s;
            L[p] = r;
            hit = true;
            break;
        }
    }
    px_count(hit, changed);
}

// Step III, PRUF form: up to rr jumps per pixel and launch.
__global__ __launch_bounds__(PX_T) void k_px_jump(Geom g, int32_t *__restrict__ L, int32_t rr,
                                                  int32_t *__restrict__ changed) {
    int32_t p;
    bool moved = false;
    if (px_index(g, p)) {
        int32_t l = L[p];
        for (int k = 0; k < rr; ++k) {
            int32_t ll = ld_par(L + l);
            if (ll == l) break;
            l = ll;
            moved = true;
        }
        if (moved) L[p] = l;
    }
    px_count(moved, changed);
}

// Step III, APRUF form (and the Find after the Step IV unions): every pixel
// follows its own chain to the root. Other threads only ever store roots into
// the chain, so a read-only chase ends at the same root.
__global__ __launch_bounds__(PX_T) void k_px_find(Geom g, int32_t *__restrict__ L) {
    int32_t p;
    if (!px_index(g, p)) return;
    int32_t l0 = L[p];
    int32_t l = gfind_ro(L, l0);
    if (l != l0) L[p] = l;
}

// Step IV, union-find form: unite the roots of adjacent minimal-plateau pixels
// (q after p only). After Step III every label is a root, and roots are only
// hooked below smaller roots, so the chased part of L is ordered.
template <int CONN>
__global__ __launch_bounds__(PX_T) void k_px_union(Geom g, const int32_t *__restrict__ S, int32_t *__restrict__ L) {
    int32_t p;
    if (!px_index(g, p) || S[p] < PX_ST2) return;
    int x, y, z;
    pixel_coords(g, p, x, y, z);
    constexpr int H = px_nnb<CONN>() / 2;
#pragma unroll
    for (int k = H; k < px_nnb<CONN>(); ++k) {
        int32_t r = px_nb<CONN>(g, p, x, y, z, k);
        if (r < 0 || S[r] < PX_ST2) continue;
        gunion(L, ld_par(L + p), ld_par(L + r));
    }
}

__device__ __forceinline__ int32_t px_ld(const int32_t *a) {
    return __hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Step IV, PRW form (Alg. 2): for adjacent minimal-plateau pixels the labels
// of their labels are lowered to the smaller of the two until they agree, then
// every pixel shortens its own label path; repeated by the host until a pass
// changes nothing. Every store is an atomic minimum, so labels only decrease
// and passes end. A thread gives up an exchange after PX_SPIN rounds and
// reports a change, which makes the host run another pass.
template <int CONN>
__global__ __launch_bounds__(PX_T) void k_px_prw(Geom g, const int32_t *__restrict__ S, int32_t *__restrict__ L,
                                                 int32_t *__restrict__ changed) {
    int32_t p;
    bool ch = false;
    if (px_index(g, p)) {
        if (S[p] >= PX_ST2) {
            int x, y, z;
            pixel_coords(g, p, x, y, z);
            constexpr int H = px_nnb<CONN>() / 2;
            for (int k = H; k < px_nnb<CONN>(); ++k) {
                int32_t r = px_nb<CONN>(g, p, x, y, z, k);
                if (r < 0 || S[r] < PX_ST2) continue;
                const int32_t lp = px_ld(L + p), lq = px_ld(L + r);
                int it = 0;
                for (; it < PX_SPIN; ++it) {
                    int32_t a = px_ld(L + lp), b = px_ld(L + lq);
                    if (a == b) break;
                    int32_t m = a < b ? a : b;
                    if (a != m) atomicMin(L + lp, m);
                    if (b != m) atomicMin(L + lq, m);
                    ch = true;
                }
                if (it == PX_SPIN) ch = true;
            }
        }
        int it = 0;
        for (; it < PX_SPIN; ++it) {
            int32_t l = px_ld(L + p), ll = px_ld(L + l);
            if (ll >= l) break;
            atomicMin(L + p, ll);
            ch = true;
        }
        if (it == PX_SPIN) ch = true;
    }
    px_count(ch, changed);
}

// Canonical labels: the smallest pixel index of every basin, gathered through
// the basin's root. M must hold 0x7fffffff everywhere before k_px_canon_min.
__global__ __launch_bounds__(PX_T) void k_px_canon_min(Geom g, const int32_t *__restrict__ L, int32_t *__restrict__ M) {
    int32_t p;
    if (!px_index(g, p)) return;
    int32_t r = L[p];
    if (p < M[r]) atomicMin(M + r, p);
}

__global__ __launch_bounds__(PX_T) void k_px_canon_apply(Geom g, int32_t *__restrict__ L, const int32_t *__restrict__ M) {
    int32_t p;
    if (!px_index(g, p)) return;
    L[p] = M[L[p]];
}

// Balanced encoding of the Step II result (ws_watershed_stages).
__global__ __launch_bounds__(PX_T) void k_px_stages(Geom g, const int32_t *__restrict__ S, int32_t *__restrict__ bal) {
    int32_t p;
    if (!px_index(g, p)) return;
    int32_t s = S[p];
    bal[p] = s == 0 ? 0 : s == PX_ST1 ? 1 : s == PX_ST2 ? 2 : s == PX_ST3 ? 3 : -s;
}

static dim3 px_grid(const Geom &g) { return dim3((uint32_t)(((int64_t)g.n + PX_T - 1) / PX_T)); }

template <int CONN, typename T>
static int px_step1_t(Launch &lc, const Geom &g, const void *I, int32_t *L, int32_t *S) {
    return lc.run("px_step1", k_px_step1<CONN, T>, px_grid(g), dim3(PX_T), g, (const T *)I, L, S);
}
template <int CONN, typename T>
static int px_sweep_t(Launch &lc, const Geom &g, const void *I, int32_t *L, int32_t *S, int32_t s, int32_t *changed) {
    return lc.run("px_sweep", k_px_sweep<CONN, T>, px_grid(g), dim3(PX_T), g, (const T *)I, L, S, s, changed);
}
template <int CONN, typename T>
static int px_union_t(Launch &lc, const Geom &g, const int32_t *S, int32_t *L) {
    return lc.run("px_union", k_px_union<CONN>, px_grid(g), dim3(PX_T), g, S, L);
}
template <int CONN, typename T>
static int px_prw_t(Launch &lc, const Geom &g, const int32_t *S, int32_t *L, int32_t *changed) {
    return lc.run("px_prw", k_px_prw<CONN>, px_grid(g), dim3(PX_T), g, S, L, changed);
}

#define PX_DISPATCH(FN, conn, u16, ...)                                                   \
    switch (conn) {                                                                       \
    case 4: return u16 ? FN<4, uint16_t>(__VA_ARGS__) : FN<4, uint8_t>(__VA_ARGS__);      \
    case 8: return u16 ? FN<8, uint16_t>(__VA_ARGS__) : FN<8, uint8_t>(__VA_ARGS__);      \
    case 6: return u16 ? FN<6, uint16_t>(__VA_ARGS__) : FN<6, uint8_t>(__VA_ARGS__);      \
    case 26: return u16 ? FN<26, uint16_t>(__VA_ARGS__) : FN<26, uint8_t>(__VA_ARGS__);   \
    default: return -1;                                                                   \
    }

int launch_px_step1(Launch &lc, const Geom &g, int conn, bool u16, const void *I, int32_t *L, int32_t *S) {
    PX_DISPATCH(px_step1_t, conn, u16, lc, g, I, L, S)
}
int launch_px_sweep(Launch &lc, const Geom &g, int conn, bool u16, const void *I, int32_t *L, int32_t *S, int32_t s,
                    int32_t *changed) {
    PX_DISPATCH(px_sweep_t, conn, u16, lc, g, I, L, S, s, changed)
}
int launch_px_union(Launch &lc, const Geom &g, int conn, const int32_t *S, int32_t *L) {
    PX_DISPATCH(px_union_t, conn, false, lc, g, S, L)
}
int launch_px_prw(Launch &lc, const Geom &g, int conn, const int32_t *S, int32_t *L, int32_t *changed) {
    PX_DISPATCH(px_prw_t, conn, false, lc, g, S, L, changed)
}
int launch_px_jump(Launch &lc, const Geom &g, int32_t *L, int32_t rr, int32_t *changed) {
    return lc.run("px_jump", k_px_jump, px_grid(g), dim3(PX_T), g, L, rr, changed);
}
int launch_px_find(Launch &lc, const Geom &g, int32_t *L) {
    return lc.run("px_find", k_px_find, px_grid(g), dim3(PX_T), g, L);
}
int launch_px_canon(Launch &lc, const Geom &g, int32_t *L, int32_t *M) {
    int rc = lc.run("px_canon_min", k_px_canon_min, px_grid(g), dim3(PX_T), g, (const int32_t *)L, M);
    if (rc) return rc;
    return lc.run("px_canon_apply", k_px_canon_apply, px_grid(g), dim3(PX_T), g, L, (const int32_t *)M);
}
int launch_px_stages(Launch &lc, const Geom &g, const int32_t *S, int32_t *bal) {
    return lc.run("px_stages", k_px_stages, px_grid(g), dim3(PX_T), g, S, bal);
}

}  // namespace wsk
