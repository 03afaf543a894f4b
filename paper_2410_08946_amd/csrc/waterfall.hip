// waterfall.hip -- gfx950 kernels of the hierarchical waterfall (Section 4).
//
// One layer step (layer k-1 -> layer k), all on the device:
//   1. key[R] = min over boundary pairs (p in R, q in N(p), q outside R) of
//      (max(I(p), I(q)) << 32) | label(q)         (Alg. 4 Step V + tie label)
//      -- a 64-bit atomicMin per run of equal labels inside a wavefront.
//   2. union(R, target(key[R])) for every region of layer k-1 (CAS hooking of
//      the larger root below the smaller, so a group's root is its smallest
//      label), then compression.
//   3. compaction of the surviving roots (the region list of layer k) and the
//      per-pixel relabel out_k[p] = root(out_{k-1}[p]).
// Region tables are indexed by label (= a pixel index), so they are N long but
// only the entries of live labels are touched.
#include "ws_device.h"
#include "ws_kernels.h"

namespace wsk {

constexpr uint64_t NOKEY = ~0ull;

// Region list of layer 0: pixels that carry their own label.
__global__ __launch_bounds__(NTHREADS) void k_wf_init(int32_t n, const int32_t *__restrict__ lab,
                                                      int32_t *__restrict__ list, int32_t *__restrict__ count,
                                                      uint64_t *__restrict__ key, int32_t *__restrict__ par) {
    int32_t p = blockIdx.x * NTHREADS + threadIdx.x;
    bool root = p < n && lab[p] == p;
    if (root) {
        key[p] = NOKEY;
        par[p] = p;
    }
    wave_append(root, p, list, count);
}

// Step V: lowest boundary pass of every region, with the label across it.
template <int CONN, typename T>
__global__ __launch_bounds__(NTHREADS) void k_wf_edge(Geom g, const T *__restrict__ I, const int32_t *__restrict__ lab,
                                                      uint64_t *__restrict__ key) {
    int32_t p = blockIdx.x * NTHREADS + threadIdx.x;
    bool valid = p < g.n;
    int32_t lp = -1;
    uint64_t best = NOKEY;
    if (valid) {
        int x, y, z;
        pixel_coords(g, p, x, y, z);
        lp = lab[p];
        uint32_t v = I[p];
#pragma unroll
        for (int k = 0; k < CONN; ++k) {
            int xx = x + nb_dx<CONN>(k), yy = y + nb_dy<CONN>(k), zz = z + nb_dz<CONN>(k);
            if (!in_image(g, xx, yy, zz)) continue;
            int32_t r = xx + g.nx * (yy + g.ny * zz);
            int32_t lq = lab[r];
            if (lq == lp) continue;
            uint32_t w = I[r];
            uint64_t c = ((uint64_t)(v > w ? v : w) << 32) | (uint32_t)lq;
            best = c < best ? c : best;
        }
    }
    // Segmented minimum over runs of equal labels in consecutive lanes; the
    // last lane of each run issues the atomic.
    int lane = __lane_id();
    int prev = __shfl_up(lp, 1);
    int head = (lane == 0 || prev != lp) ? lane : 0;
    int rs = head;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        int t = __shfl_up(rs, off);
        if (lane >= off && t > rs) rs = t;
    }
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint64_t t = __shfl_up(best, off);
        if (lane - off >= rs && t < best) best = t;
    }
    int next = __shfl_down(lp, 1);
    bool tail = lane == 63 || next != lp;
    if (valid && tail && best != NOKEY) atomicMin((unsigned long long *)(key + lp), (unsigned long long)best);
}

// Join every region with the region across its lowest pass.
__global__ __launch_bounds__(NTHREADS) void k_wf_union(const int32_t *__restrict__ list,
                                                       const int32_t *__restrict__ count,
                                                       const uint64_t *__restrict__ key, int32_t *__restrict__ par) {
    int32_t c = *count;
    for (int32_t i = blockIdx.x * NTHREADS + threadIdx.x; i < c; i += gridDim.x * NTHREADS) {
        int32_t r = list[i];
        uint64_t kk = key[r];
        if (kk != NOKEY) gunion(par, r, (int32_t)(uint32_t)(kk & 0xffffffffull));
    }
}

__global__ __launch_bounds__(NTHREADS) void k_wf_compress(const int32_t *__restrict__ list,
                                                          const int32_t *__restrict__ count,
                                                          int32_t *__restrict__ par) {
    int32_t c = *count;
    for (int32_t i = blockIdx.x * NTHREADS + threadIdx.x; i < c; i += gridDim.x * NTHREADS) {
        int32_t r = list[i];
        par[r] = gfind_ro(par, r);
    }
}

// Surviving roots form the next region list; their keys are reset.
__global__ __launch_bounds__(NTHREADS) void k_wf_compact(const int32_t *__restrict__ list_in,
                                                         const int32_t *__restrict__ count_in,
                                                         int32_t *__restrict__ list_out,
                                                         int32_t *__restrict__ count_out,
                                                         const int32_t *__restrict__ par,
                                                         uint64_t *__restrict__ key) {
    int32_t c = *count_in;
    int32_t stride = gridDim.x * NTHREADS;
    for (int32_t base = blockIdx.x * NTHREADS; base < c; base += stride) {
        int32_t i = base + threadIdx.x;
        bool root = false;
        int32_t r = 0;
        if (i < c) {
            r = list_in[i];
            root = par[r] == r;
            if (root) key[r] = NOKEY;
        }
        wave_append(root, r, list_out, count_out);
    }
}

__global__ __launch_bounds__(NTHREADS) void k_wf_relabel(int32_t n, const int32_t *__restrict__ prev,
                                                         int32_t *__restrict__ cur, const int32_t *__restrict__ par) {
    int32_t p = blockIdx.x * NTHREADS + threadIdx.x;
    if (p < n) cur[p] = par[prev[p]];
}

__global__ void k_wf_counts(int32_t nl, const int32_t *__restrict__ counts, int64_t *__restrict__ out) {
    for (int i = threadIdx.x; i < nl; i += blockDim.x) out[i] = counts[i];
}

// ---------------------------------------------------------------------------
template <int CONN, typename T>
static int launch_wf_edge_t(Launch &lc, const Geom &g, const void *I, const int32_t *lab, uint64_t *key) {
    return lc.run("wf_edge", k_wf_edge<CONN, T>, dim3((g.n + NTHREADS - 1) / NTHREADS), dim3(NTHREADS), g,
                  (const T *)I, lab, key);
}

int launch_wf_edge(Launch &lc, const Geom &g, int conn, bool u16, const void *I, const int32_t *lab, uint64_t *key) {
    switch (conn) {
    case 4: return u16 ? launch_wf_edge_t<4, uint16_t>(lc, g, I, lab, key) : launch_wf_edge_t<4, uint8_t>(lc, g, I, lab, key);
    case 8: return u16 ? launch_wf_edge_t<8, uint16_t>(lc, g, I, lab, key) : launch_wf_edge_t<8, uint8_t>(lc, g, I, lab, key);
    case 6: return u16 ? launch_wf_edge_t<6, uint16_t>(lc, g, I, lab, key) : launch_wf_edge_t<6, uint8_t>(lc, g, I, lab, key);
    case 26: return u16 ? launch_wf_edge_t<26, uint16_t>(lc, g, I, lab, key) : launch_wf_edge_t<26, uint8_t>(lc, g, I, lab, key);
    default: return -1;
    }
}

static inline dim3 list_grid(int32_t n) {
    int32_t b = (n + NTHREADS - 1) / NTHREADS;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    return dim3(b);
}

int launch_wf_init(Launch &lc, int32_t n, const int32_t *lab, int32_t *list, int32_t *count, uint64_t *key, int32_t *par) {
    return lc.run("wf_init", k_wf_init, dim3((n + NTHREADS - 1) / NTHREADS), dim3(NTHREADS), n, lab, list, count, key, par);
}
int launch_wf_union(Launch &lc, int32_t bound, const int32_t *list, const int32_t *count, const uint64_t *key, int32_t *par) {
    return lc.run("wf_union", k_wf_union, list_grid(bound), dim3(NTHREADS), list, count, key, par);
}
int launch_wf_compress(Launch &lc, int32_t bound, const int32_t *list, const int32_t *count, int32_t *par) {
    return lc.run("wf_compress", k_wf_compress, list_grid(bound), dim3(NTHREADS), list, count, par);
}
int launch_wf_compact(Launch &lc, int32_t bound, const int32_t *list_in, const int32_t *count_in, int32_t *list_out,
                      int32_t *count_out, const int32_t *par, uint64_t *key) {
    return lc.run("wf_compact", k_wf_compact, list_grid(bound), dim3(NTHREADS), list_in, count_in, list_out, count_out,
                  par, key);
}
int launch_wf_relabel(Launch &lc, int32_t n, const int32_t *prev, int32_t *cur, const int32_t *par) {
    return lc.run("wf_relabel", k_wf_relabel, dim3((n + NTHREADS - 1) / NTHREADS), dim3(NTHREADS), n, prev, cur, par);
}
int launch_wf_counts(Launch &lc, int32_t nl, const int32_t *counts, int64_t *out) {
    return lc.run("wf_counts", k_wf_counts, dim3(1), dim3(256), nl, counts, out);
}

}  // namespace wsk
