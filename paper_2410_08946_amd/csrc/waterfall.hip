// waterfall.hip -- gfx950 kernels of the hierarchical waterfall (Section 4).
//
// One layer step (layer k-1 -> layer k), all on the device:
//   1. key[R] = min over boundary pairs (p in R, q in N(p), q outside R) of
//      (max(I(p), I(q)) << 32) | label(q)         (Alg. 4 Step V + tie label)
//      computed per tile: per-pixel candidates are reduced per label in an LDS
//      hash table (64-bit LDS atomic min), then one global atomicMin per
//      (tile, label), skipped when the global key is already smaller.
//   2. union(R, target(key[R])) for every region of layer k-1 (CAS hooking of
//      the larger root below the smaller, so a group's root is its smallest
//      label), then compression to the root.
//   3. compaction of the surviving roots into the region list of layer k.
// The relabel out_k[p] = root(out_{k-1}[p]) is done by the next layer's key
// kernel while it loads its labels (and by a last pass for the final layer).
// Region tables are indexed by label (= a pixel index), so they are N long but
// only the entries of live labels are touched.
#include "ws_device.h"
#include "ws_kernels.h"

namespace wsk {

constexpr uint64_t NOKEY = ~0ull;

// ---------------------------------------------------------------------------
// Order-preserving compaction in three kernels (no contended atomics):
// per-chunk counts, one-block exclusive scan, per-chunk ordered writes.
// Source 0: pixels p < n with lab[p] == p (layer-0 regions; also initialises
// key[p] and par[p]). Source 1: list entries r with par[r] == r (survivors;
// also resets key[r]).
// ---------------------------------------------------------------------------
constexpr int CITEMS = 16;                      // elements per thread per chunk
constexpr int CCHUNK = NTHREADS * CITEMS;       // elements per chunk

struct CompactSrc {
    int mode;                     // 0 = pixels, 1 = list
    int32_t n;                    // mode 0: number of pixels
    const int32_t *lab;           // mode 0
    const int32_t *list;          // mode 1
    const int32_t *count;         // mode 1: device count of list
    const int32_t *par;           // mode 1
};

__device__ __forceinline__ int32_t src_size(const CompactSrc &s) { return s.mode == 0 ? s.n : *s.count; }

// Predicates and values of CITEMS elements (element j at first + j * step),
// with all loads of a phase issued before any is used.
__device__ __forceinline__ uint32_t src_batch(const CompactSrc &s, int32_t n, int32_t first, int32_t step,
                                              int32_t *vals) {
    int32_t a[CITEMS];
    uint32_t in = 0;
#pragma unroll
    for (int j = 0; j < CITEMS; ++j) {
        int32_t i = first + j * step;
        if (i < n) in |= 1u << j;
        a[j] = s.mode == 0 ? s.lab[i < n ? i : 0] : s.list[i < n ? i : 0];
    }
    uint32_t mask = 0;
    if (s.mode == 0) {
#pragma unroll
        for (int j = 0; j < CITEMS; ++j) {
            int32_t i = first + j * step;
            vals[j] = i;
            if ((in >> j & 1u) && a[j] == i) mask |= 1u << j;
        }
    } else {
        int32_t b[CITEMS];
#pragma unroll
        for (int j = 0; j < CITEMS; ++j) b[j] = s.par[a[j]];
#pragma unroll
        for (int j = 0; j < CITEMS; ++j) {
            vals[j] = a[j];
            if ((in >> j & 1u) && b[j] == a[j]) mask |= 1u << j;
        }
    }
    return mask;
}

// Block-wide exclusive scan of one int per thread; returns the block total.
__device__ __forceinline__ int block_scan_excl(int v, int &excl) {
    __shared__ int wsum[NTHREADS / 64];
    int lane = __lane_id(), w = threadIdx.x >> 6;
    int x = v;
    for (int off = 1; off < 64; off <<= 1) {
        int t = __shfl_up(x, off);
        if (lane >= off) x += t;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    int base = 0, total = 0;
    for (int k = 0; k < NTHREADS / 64; ++k) {
        if (k < w) base += wsum[k];
        total += wsum[k];
    }
    excl = base + x - v;
    __syncthreads();
    return total;
}

__global__ __launch_bounds__(NTHREADS) void k_compact_count(CompactSrc s, int32_t *__restrict__ chunk_count) {
    int32_t n = src_size(s);
    int32_t nchunks = (n + CCHUNK - 1) / CCHUNK;
    for (int32_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        int32_t vals[CITEMS];
        int cnt = __popc(src_batch(s, n, c * CCHUNK + threadIdx.x, NTHREADS, vals));
        int excl;
        int total = block_scan_excl(cnt, excl);
        if (threadIdx.x == 0) chunk_count[c] = total;
    }
}

// Exclusive scan of the chunk counts in place (one workgroup); writes the
// total into *count_out.
__global__ __launch_bounds__(NTHREADS) void k_compact_scan(CompactSrc s, int32_t *__restrict__ chunk_count,
                                                           int32_t *__restrict__ count_out) {
    int32_t n = src_size(s);
    int32_t nchunks = (n + CCHUNK - 1) / CCHUNK;
    int32_t carry = 0;
    for (int32_t base = 0; base < nchunks; base += NTHREADS) {
        int32_t i = base + threadIdx.x;
        int v = i < nchunks ? chunk_count[i] : 0;
        int excl;
        int total = block_scan_excl(v, excl);
        if (i < nchunks) chunk_count[i] = carry + excl;
        carry += total;
    }
    if (threadIdx.x == 0) *count_out = carry;
}

__global__ __launch_bounds__(NTHREADS) void k_compact_write(CompactSrc s, const int32_t *__restrict__ chunk_off,
                                                            int32_t *__restrict__ list_out, uint64_t *__restrict__ key,
                                                            int32_t *__restrict__ par_init) {
    int32_t n = src_size(s);
    int32_t nchunks = (n + CCHUNK - 1) / CCHUNK;
    for (int32_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        // per thread: its elements are a contiguous run of CITEMS inside the
        // chunk, so the written order equals the source order
        int32_t vals[CITEMS];
        uint32_t mask = src_batch(s, n, c * CCHUNK + threadIdx.x * CITEMS, 1, vals);
        int excl;
        block_scan_excl(__popc(mask), excl);
        int32_t o = chunk_off[c] + excl;
        for (int j = 0; j < CITEMS; ++j) {
            if (!(mask & (1u << j))) continue;
            int32_t r = vals[j];
            list_out[o++] = r;
            key[r] = NOKEY;
            if (par_init) par_init[r] = r;
        }
    }
}

// ---------------------------------------------------------------------------
// Step V per tile with LDS aggregation; optionally maps the labels it loads
// through `map` (the previous layer's roots) and writes the mapped labels of
// its own pixels to `cur` (the relabel of the previous layer).
// ---------------------------------------------------------------------------
template <int NDIM> struct WfTile;
template <> struct WfTile<2> { static constexpr int X = 64, Y = 16, Z = 1; };
template <> struct WfTile<3> { static constexpr int X = 16, Y = 8, Z = 8; };
constexpr int HSLOTS = 1024;  // LDS hash slots (>= pixels per tile, so probing ends)
constexpr int HBITS = 10;

template <int CONN, typename T>
__global__ __launch_bounds__(NTHREADS) void k_wf_edge(Geom g, const T *__restrict__ I, const int32_t *__restrict__ prev,
                                                      const int32_t *__restrict__ map, int32_t *__restrict__ cur,
                                                      uint64_t *__restrict__ key) {
    constexpr int NDIM = ndim_of<CONN>();
    using TS = WfTile<NDIM>;
    constexpr int SX = TS::X + 2, SY = TS::Y + 2, SZ = NDIM == 3 ? TS::Z + 2 : 1, RZ = NDIM == 3 ? 1 : 0;
    constexpr int CELLS = SX * SY * SZ;
    constexpr int PIX = TS::X * TS::Y * TS::Z;
    __shared__ int sL[CELLS];
    __shared__ int sI[CELLS];
    __shared__ int hk[HSLOTS];
    __shared__ unsigned long long hv[HSLOTS];
    int ntx = (g.nx + TS::X - 1) / TS::X, nty = (g.ny + TS::Y - 1) / TS::Y;
    int t = blockIdx.x;
    int ox = (t % ntx) * TS::X, oy = ((t / ntx) % nty) * TS::Y, oz = (t / (ntx * nty)) * TS::Z;
    {
        // batched loads: labels and grey values first, then the label map
        constexpr int PER = (CELLS + NTHREADS - 1) / NTHREADS;
        int32_t idx[PER];
        bool ok[PER], inner[PER];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            int c = threadIdx.x + j * NTHREADS;
            int cx = c % SX, cy = (c / SX) % SY, cz = c / (SX * SY);
            int x = ox + cx - 1, y = oy + cy - 1, z = oz + cz - RZ;
            ok[j] = c < CELLS && in_image(g, x, y, z);
            inner[j] = cx >= 1 && cx <= TS::X && cy >= 1 && cy <= TS::Y && (NDIM == 2 || (cz >= 1 && cz <= TS::Z));
            idx[j] = ok[j] ? x + g.nx * (y + g.ny * z) : 0;
        }
        int32_t lv[PER];
        T gv[PER];
#pragma unroll
        for (int j = 0; j < PER; ++j) lv[j] = prev[idx[j]];
#pragma unroll
        for (int j = 0; j < PER; ++j) gv[j] = I[idx[j]];
        if (map) {
#pragma unroll
            for (int j = 0; j < PER; ++j) lv[j] = map[lv[j]];
#pragma unroll
            for (int j = 0; j < PER; ++j)
                if (ok[j] && inner[j]) cur[idx[j]] = lv[j];
        }
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            int c = threadIdx.x + j * NTHREADS;
            if (c < CELLS) {
                sL[c] = ok[j] ? lv[j] : -1;
                sI[c] = ok[j] ? (int)gv[j] : SENT;
            }
        }
    }
    for (int h = threadIdx.x; h < HSLOTS; h += NTHREADS) {
        hk[h] = -1;
        hv[h] = NOKEY;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < PIX; i += NTHREADS) {
        int x = i % TS::X, y = (i / TS::X) % TS::Y, z = i / (TS::X * TS::Y);
        int s = ((z + RZ) * SY + (y + 1)) * SX + (x + 1);
        int l = sL[s];
        if (l < 0) continue;
        uint32_t v = (uint32_t)sI[s];
        uint64_t best = NOKEY;
#pragma unroll
        for (int k = 0; k < CONN; ++k) {
            int o = s + nb_dx<CONN>(k) + SX * (nb_dy<CONN>(k) + SY * nb_dz<CONN>(k));
            int lq = sL[o];
            if (lq < 0 || lq == l) continue;
            uint32_t w = (uint32_t)sI[o];
            uint64_t c = ((uint64_t)(v > w ? v : w) << 32) | (uint32_t)lq;
            best = c < best ? c : best;
        }
        if (best == NOKEY) continue;
        uint32_t h = ((uint32_t)l * 2654435761u) >> (32 - HBITS);
        for (;;) {
            int old = atomicCAS(&hk[h], -1, l);
            if (old == -1 || old == l) {
                atomicMin(&hv[h], (unsigned long long)best);
                break;
            }
            h = (h + 1) & (HSLOTS - 1);
        }
    }
    __syncthreads();
    for (int h = threadIdx.x; h < HSLOTS; h += NTHREADS) {
        int l = hk[h];
        if (l < 0) continue;
        atomicMin((unsigned long long *)(key + l), hv[h]);
    }
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
static int launch_wf_edge_t(Launch &lc, const Geom &g, const void *I, const int32_t *prev, const int32_t *map,
                            int32_t *cur, uint64_t *key) {
    constexpr int ND = ndim_of<CONN>();
    using TS = WfTile<ND>;
    int tiles = ((g.nx + TS::X - 1) / TS::X) * ((g.ny + TS::Y - 1) / TS::Y) * ((g.nz + TS::Z - 1) / TS::Z);
    return lc.run("wf_edge", k_wf_edge<CONN, T>, dim3(tiles), dim3(NTHREADS), g, (const T *)I, prev, map, cur, key);
}

int launch_wf_edge(Launch &lc, const Geom &g, int conn, bool u16, const void *I, const int32_t *prev,
                   const int32_t *map, int32_t *cur, uint64_t *key) {
    switch (conn) {
    case 4: return u16 ? launch_wf_edge_t<4, uint16_t>(lc, g, I, prev, map, cur, key) : launch_wf_edge_t<4, uint8_t>(lc, g, I, prev, map, cur, key);
    case 8: return u16 ? launch_wf_edge_t<8, uint16_t>(lc, g, I, prev, map, cur, key) : launch_wf_edge_t<8, uint8_t>(lc, g, I, prev, map, cur, key);
    case 6: return u16 ? launch_wf_edge_t<6, uint16_t>(lc, g, I, prev, map, cur, key) : launch_wf_edge_t<6, uint8_t>(lc, g, I, prev, map, cur, key);
    case 26: return u16 ? launch_wf_edge_t<26, uint16_t>(lc, g, I, prev, map, cur, key) : launch_wf_edge_t<26, uint8_t>(lc, g, I, prev, map, cur, key);
    default: return -1;
    }
}

static inline dim3 list_grid(int32_t n) {
    int32_t b = (n + NTHREADS - 1) / NTHREADS;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    return dim3(b);
}

static inline dim3 chunk_grid(int32_t bound) {
    int32_t c = (bound + CCHUNK - 1) / CCHUNK;
    if (c > 4096) c = 4096;
    if (c < 1) c = 1;
    return dim3(c);
}

int compact_chunks(int32_t bound) { return (bound + CCHUNK - 1) / CCHUNK; }

// Compaction of layer-0 regions (pixels with lab[p] == p).
int launch_wf_init(Launch &lc, int32_t n, const int32_t *lab, int32_t *list, int32_t *count, uint64_t *key, int32_t *par,
                   int32_t *chunk_tmp) {
    CompactSrc s{0, n, lab, nullptr, nullptr, nullptr};
    int rc = lc.run("wf_init", k_compact_count, chunk_grid(n), dim3(NTHREADS), s, chunk_tmp);
    if (rc) return rc;
    rc = lc.run("wf_init", k_compact_scan, dim3(1), dim3(NTHREADS), s, chunk_tmp, count);
    if (rc) return rc;
    return lc.run("wf_init", k_compact_write, chunk_grid(n), dim3(NTHREADS), s, (const int32_t *)chunk_tmp, list, key, par);
}

// Compaction of surviving roots of a region list.
int launch_wf_compact(Launch &lc, int32_t bound, const int32_t *list_in, const int32_t *count_in, int32_t *list_out,
                      int32_t *count_out, const int32_t *par, uint64_t *key, int32_t *chunk_tmp) {
    CompactSrc s{1, 0, nullptr, list_in, count_in, par};
    int rc = lc.run("wf_compact", k_compact_count, chunk_grid(bound), dim3(NTHREADS), s, chunk_tmp);
    if (rc) return rc;
    rc = lc.run("wf_compact", k_compact_scan, dim3(1), dim3(NTHREADS), s, chunk_tmp, count_out);
    if (rc) return rc;
    return lc.run("wf_compact", k_compact_write, chunk_grid(bound), dim3(NTHREADS), s, (const int32_t *)chunk_tmp, list_out,
                  key, (int32_t *)nullptr);
}

int launch_wf_union(Launch &lc, int32_t bound, const int32_t *list, const int32_t *count, const uint64_t *key, int32_t *par) {
    return lc.run("wf_union", k_wf_union, list_grid(bound), dim3(NTHREADS), list, count, key, par);
}
int launch_wf_compress(Launch &lc, int32_t bound, const int32_t *list, const int32_t *count, int32_t *par) {
    return lc.run("wf_compress", k_wf_compress, list_grid(bound), dim3(NTHREADS), list, count, par);
}
int launch_wf_relabel(Launch &lc, int32_t n, const int32_t *prev, int32_t *cur, const int32_t *par) {
    return lc.run("wf_relabel", k_wf_relabel, dim3((n + NTHREADS - 1) / NTHREADS), dim3(NTHREADS), n, prev, cur, par);
}
int launch_wf_counts(Launch &lc, int32_t nl, const int32_t *counts, int64_t *out) {
    return lc.run("wf_counts", k_wf_counts, dim3(1), dim3(256), nl, counts, out);
}

}  // namespace wsk
