// waterfall.hip -- gfx950 kernels of the hierarchical waterfall (Section 4).
//
// One layer step (layer k-1 -> layer k), all on the device:
//   1. key[R] = min over boundary pairs (p in R, q in N(p), q outside R) of
//      (max(I(p), I(q)) << 32) | label(q)         (Alg. 4 Step V + tie label)
//      computed per tile: per-pixel candidates are reduced per label in an LDS
//      hash table (64-bit LDS atomic min), then one global atomicMin per
//      (tile, label).
//   2. union(R, target(key[R])) for every region of layer k-1 (CAS hooking of
//      the larger root below the smaller, so a group's root is its smallest
//      label), then compression to the root.
//   3. compaction of the surviving roots into the region list of layer k.
// The relabel out_k[p] = root(out_{k-1}[p]) is done by the next layer's key
// kernel while it loads its labels (and by a last pass for the final layer),
// which also counts each tile's regions (pixels carrying their own label).
//
// Region tables (keys, parents, lists) use arena labels: the image's arena
// offset plus its local canonical label, so the region-level kernels need no
// image lookup and images of a batch never interact. The tables are indexed by
// label, so they are arena-long but only the entries of live labels are used.
#include "ws_device.h"
#include "ws_kernels.h"

namespace wsk {

constexpr uint64_t NOKEY = ~0ull;

template <int NDIM> struct WfTile;
template <> struct WfTile<2> { static constexpr int X = 64, Y = 16, Z = 1; };
template <> struct WfTile<3> { static constexpr int X = 16, Y = 8, Z = 8; };
constexpr int HSLOTS = 1024;  // LDS hash slots (>= pixels per tile, so probing ends)
constexpr int HBITS = 10;

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

// ---------------------------------------------------------------------------
// Layer-0 region lists: per tile, the pixels that carry their own label, in
// tile order then pixel order; written as arena labels. Also initialises
// their keys and parents. Per-tile counts are kept for per-image counts.
// ---------------------------------------------------------------------------
template <int NDIM, class Src>
__global__ __launch_bounds__(NTHREADS) void k_root_count(Src src, int32_t ntiles, int32_t *__restrict__ tile_cnt,
                                                         int32_t *__restrict__ tile_cnt_keep) {
    using TS = WfTile<NDIM>;
    constexpr int PER = TS::X * TS::Y * TS::Z / NTHREADS;
    {
        const int t = blockIdx.x;
        if (t >= ntiles) return;
        Img im;
        int lt;
        fetch(src, t, TK_WF, im, lt);
        const Geom &g = im.g;
        int ox, oy, oz;
        tile_xyz<TS::X, TS::Y, TS::Z>(g, lt, ox, oy, oz);
        int32_t p[PER], l[PER];
        bool ok[PER];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            int i = threadIdx.x * PER + j;
            int x = ox + i % TS::X, y = oy + (i / TS::X) % TS::Y, z = oz + i / (TS::X * TS::Y);
            ok[j] = in_image(g, x, y, z);
            p[j] = ok[j] ? x + g.nx * (y + g.ny * z) : 0;
        }
#pragma unroll
        for (int j = 0; j < PER; ++j) l[j] = im.lab[p[j]];
        int cnt = 0;
#pragma unroll
        for (int j = 0; j < PER; ++j) cnt += (ok[j] && l[j] == p[j]) ? 1 : 0;
        int excl;
        int total = block_scan_excl(cnt, excl);
        if (threadIdx.x == 0) {
            tile_cnt[t] = total;
            tile_cnt_keep[t] = total;
        }
    }
}

template <int NDIM, class Src>
__global__ __launch_bounds__(NTHREADS) void k_root_write(Src src, int32_t ntiles, const int32_t *__restrict__ tile_off,
                                                         int32_t *__restrict__ list, uint64_t *__restrict__ key,
                                                         int32_t *__restrict__ par) {
    using TS = WfTile<NDIM>;
    constexpr int PER = TS::X * TS::Y * TS::Z / NTHREADS;
    {
        const int t = blockIdx.x;
        if (t >= ntiles) return;
        Img im;
        int lt;
        fetch(src, t, TK_WF, im, lt);
        const Geom &g = im.g;
        int ox, oy, oz;
        tile_xyz<TS::X, TS::Y, TS::Z>(g, lt, ox, oy, oz);
        int32_t p[PER], l[PER];
        bool ok[PER];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            int i = threadIdx.x * PER + j;
            int x = ox + i % TS::X, y = oy + (i / TS::X) % TS::Y, z = oz + i / (TS::X * TS::Y);
            ok[j] = in_image(g, x, y, z);
            p[j] = ok[j] ? x + g.nx * (y + g.ny * z) : 0;
        }
#pragma unroll
        for (int j = 0; j < PER; ++j) l[j] = im.lab[p[j]];
        uint32_t mask = 0;
#pragma unroll
        for (int j = 0; j < PER; ++j)
            if (ok[j] && l[j] == p[j]) mask |= 1u << j;
        int excl;
        block_scan_excl(__popc(mask), excl);
        int32_t o = tile_off[t] + excl;
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            if (!(mask >> j & 1u)) continue;
            int32_t G = im.pix0 + p[j];
            list[o++] = G;
            key[G] = NOKEY;
            par[G] = G;
        }
    }
}

// ---------------------------------------------------------------------------
// Order-preserving compaction of a region list (survivors: par[r] == r) in
// three kernels without contended atomics: per-chunk counts, a one-workgroup
// exclusive scan, per-chunk ordered writes (which also reset the keys).
// ---------------------------------------------------------------------------
constexpr int CITEMS = 16;                      // elements per thread per chunk
constexpr int CCHUNK = NTHREADS * CITEMS;       // elements per chunk

// Predicates and values of CITEMS list elements (element j at first + j*step),
// with all loads of a phase issued before any is used.
__device__ __forceinline__ uint32_t list_batch(const int32_t *__restrict__ list, const int32_t *__restrict__ par,
                                               int32_t n, int32_t first, int32_t step, int32_t *vals) {
    int32_t a[CITEMS], b[CITEMS];
    uint32_t in = 0;
#pragma unroll
    for (int j = 0; j < CITEMS; ++j) {
        int32_t i = first + j * step;
        if (i < n) in |= 1u << j;
        a[j] = list[i < n ? i : 0];
    }
#pragma unroll
    for (int j = 0; j < CITEMS; ++j) b[j] = par[a[j]];
    uint32_t mask = 0;
#pragma unroll
    for (int j = 0; j < CITEMS; ++j) {
        vals[j] = a[j];
        if ((in >> j & 1u) && b[j] == a[j]) mask |= 1u << j;
    }
    return mask;
}

__global__ __launch_bounds__(NTHREADS) void k_compact_count(const int32_t *__restrict__ list,
                                                            const int32_t *__restrict__ count,
                                                            const int32_t *__restrict__ par,
                                                            int32_t *__restrict__ chunk_count) {
    int32_t n = *count;
    int32_t nchunks = (n + CCHUNK - 1) / CCHUNK;
    for (int32_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        int32_t vals[CITEMS];
        int cnt = __popc(list_batch(list, par, n, c * CCHUNK + threadIdx.x, NTHREADS, vals));
        int excl;
        int total = block_scan_excl(cnt, excl);
        if (threadIdx.x == 0) chunk_count[c] = total;
    }
}

// Exclusive scan of n counts in place (one workgroup); total into *total_out.
// n is derived from *n_dev when given (chunks of a device-sized list). Each
// thread owns a contiguous run of the counts (loads issued together), the
// runs' sums are scanned across the workgroup, then each run is rewritten.
__global__ __launch_bounds__(NTHREADS) void k_scan(int32_t n_host, const int32_t *__restrict__ n_dev, int32_t chunk,
                                                   int32_t *__restrict__ cnt, int32_t *__restrict__ total_out) {
    constexpr int U = 16;
    int32_t n = n_dev ? (*n_dev + chunk - 1) / chunk : n_host;
    int32_t per = (n + NTHREADS - 1) / NTHREADS;
    int32_t lo = threadIdx.x * per, hi = lo + per < n ? lo + per : n;
    int32_t sum = 0;
    for (int32_t b = lo; b < hi; b += U) {
        int32_t v[U];
#pragma unroll
        for (int j = 0; j < U; ++j) v[j] = b + j < hi ? cnt[b + j] : 0;
#pragma unroll
        for (int j = 0; j < U; ++j) sum += v[j];
    }
    int excl;
    int total = block_scan_excl(sum, excl);
    int32_t run = excl;
    for (int32_t b = lo; b < hi; b += U) {
        int32_t v[U];
#pragma unroll
        for (int j = 0; j < U; ++j) v[j] = b + j < hi ? cnt[b + j] : 0;
#pragma unroll
        for (int j = 0; j < U; ++j)
            if (b + j < hi) {
                cnt[b + j] = run;
                run += v[j];
            }
    }
    if (threadIdx.x == 0 && total_out) *total_out = total;
}

__global__ __launch_bounds__(NTHREADS) void k_compact_write(const int32_t *__restrict__ list,
                                                            const int32_t *__restrict__ count,
                                                            const int32_t *__restrict__ par,
                                                            const int32_t *__restrict__ chunk_off,
                                                            int32_t *__restrict__ list_out,
                                                            uint64_t *__restrict__ key) {
    int32_t n = *count;
    int32_t nchunks = (n + CCHUNK - 1) / CCHUNK;
    for (int32_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        // per thread: a contiguous run of CITEMS elements, so the written
        // order equals the source order
        int32_t vals[CITEMS];
        uint32_t mask = list_batch(list, par, n, c * CCHUNK + threadIdx.x * CITEMS, 1, vals);
        int excl;
        block_scan_excl(__popc(mask), excl);
        int32_t o = chunk_off[c] + excl;
#pragma unroll
        for (int j = 0; j < CITEMS; ++j) {
            if (!(mask >> j & 1u)) continue;
            int32_t r = vals[j];
            list_out[o++] = r;
            key[r] = NOKEY;
        }
    }
}

// ---------------------------------------------------------------------------
// Step V per tile with LDS aggregation. Layer `layer` is loaded; with
// `relabel` set its labels are first mapped through the roots in `par` (the
// merge that produced layer+1), layer+1 is written for the tile's own pixels
// and its regions are counted into tile_cnt; the keys are then those of
// layer+1 (else of `layer`).
// ---------------------------------------------------------------------------
template <int CONN, typename T, class Src>
__global__ __launch_bounds__(NTHREADS) void k_wf_edge(Src src, int32_t ntiles, int32_t layer, int32_t relabel,
                                                      const int32_t *__restrict__ par, uint64_t *__restrict__ key,
                                                      int32_t *__restrict__ tile_cnt) {
    constexpr int NDIM = ndim_of<CONN>();
    using TS = WfTile<NDIM>;
    constexpr int SX = TS::X + 2, SY = TS::Y + 2, SZ = NDIM == 3 ? TS::Z + 2 : 1, RZ = NDIM == 3 ? 1 : 0;
    constexpr int CELLS = SX * SY * SZ;
    constexpr int PIX = TS::X * TS::Y * TS::Z;
    __shared__ int sL[CELLS];
    __shared__ int sI[CELLS];
    __shared__ int hk[HSLOTS];
    __shared__ unsigned long long hv[HSLOTS];
    {
        const int t = blockIdx.x;
        if (t >= ntiles) return;
        Img im;
        int lt;
        fetch(src, t, TK_WF, im, lt);
        const Geom &g = im.g;
        const T *I = (const T *)im.grey;
        const int32_t *prev = im.lab + (size_t)layer * g.n;
        int32_t *cur = im.lab + (size_t)(layer + 1) * g.n;
        int ox, oy, oz;
        tile_xyz<TS::X, TS::Y, TS::Z>(g, lt, ox, oy, oz);
        int nroots = 0;
        {
            // batched loads: labels and grey values first, then the root map
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
            if (relabel) {
#pragma unroll
                for (int j = 0; j < PER; ++j) lv[j] = par[im.pix0 + lv[j]] - im.pix0;
#pragma unroll
                for (int j = 0; j < PER; ++j)
                    if (ok[j] && inner[j]) {
                        cur[idx[j]] = lv[j];
                        nroots += lv[j] == idx[j] ? 1 : 0;
                    }
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
        static_assert(PIX % NTHREADS == 0, "whole waves per tile");
        for (int i = threadIdx.x; i < PIX; i += NTHREADS) {  // uniform trip count
            int x = i % TS::X, y = (i / TS::X) % TS::Y, z = i / (TS::X * TS::Y);
            int s = ((z + RZ) * SY + (y + 1)) * SX + (x + 1);
            int l = sL[s];
            uint64_t best = NOKEY;
            if (l >= 0) {
                uint32_t v = (uint32_t)sI[s];
#pragma unroll
                for (int k = 0; k < CONN; ++k) {
                    int o = s + nb_dx<CONN>(k) + SX * (nb_dy<CONN>(k) + SY * nb_dz<CONN>(k));
                    int lq = sL[o];
                    if (lq < 0 || lq == l) continue;
                    uint32_t w = (uint32_t)sI[o];
                    uint64_t c = ((uint64_t)(v > w ? v : w) << 32) | (uint32_t)(im.pix0 + lq);
                    best = c < best ? c : best;
                }
            }
            if (best == NOKEY) continue;
            uint32_t h = ((uint32_t)l * 2654435761u) >> (32 - HBITS);
            for (;;) {
                int cur = hk[h];
                if (cur == -1) cur = atomicCAS(&hk[h], -1, l);
                if (cur == -1 || cur == l) {
                    atomicMin(&hv[h], (unsigned long long)best);
                    break;
                }
                h = (h + 1) & (HSLOTS - 1);
            }
        }
        __syncthreads();
        for (int h = threadIdx.x; h < HSLOTS; h += NTHREADS) {
            int l = hk[h];
            if (l >= 0) atomicMin((unsigned long long *)(key + im.pix0 + l), hv[h]);
        }
        if (relabel) {
            int excl;
            int total = block_scan_excl(nroots, excl);
            if (threadIdx.x == 0) tile_cnt[t] = total;
        }
        __syncthreads();
    }
}

// Join every region with the region across its lowest pass. The list holds
// every layer-0 region; exactly the regions of the current layer that have a
// boundary carry a key (dead regions had theirs reset when they merged), and
// each key is reset here for the next layer.
__global__ __launch_bounds__(NTHREADS) void k_wf_union(const int32_t *__restrict__ list,
                                                       const int32_t *__restrict__ count,
                                                       uint64_t *__restrict__ key, int32_t *__restrict__ par) {
    int32_t c = *count;
    for (int32_t i = blockIdx.x * NTHREADS + threadIdx.x; i < c; i += gridDim.x * NTHREADS) {
        int32_t r = list[i];
        uint64_t kk = key[r];
        if (kk == NOKEY) continue;
        key[r] = NOKEY;
        gunion(par, r, (int32_t)(uint32_t)(kk & 0xffffffffull));
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

// Last layer: out_{layer+1} = root(out_layer), with per-tile region counts.
template <int NDIM, class Src>
__global__ __launch_bounds__(NTHREADS) void k_wf_relabel(Src src, int32_t ntiles, int32_t layer,
                                                         const int32_t *__restrict__ par,
                                                         int32_t *__restrict__ tile_cnt) {
    using TS = WfTile<NDIM>;
    constexpr int PER = TS::X * TS::Y * TS::Z / NTHREADS;
    {
        const int t = blockIdx.x;
        if (t >= ntiles) return;
        Img im;
        int lt;
        fetch(src, t, TK_WF, im, lt);
        const Geom &g = im.g;
        const int32_t *prev = im.lab + (size_t)layer * g.n;
        int32_t *cur = im.lab + (size_t)(layer + 1) * g.n;
        int ox, oy, oz;
        tile_xyz<TS::X, TS::Y, TS::Z>(g, lt, ox, oy, oz);
        int32_t p[PER], l[PER];
        bool ok[PER];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            int i = threadIdx.x + j * NTHREADS;
            int x = ox + i % TS::X, y = oy + (i / TS::X) % TS::Y, z = oz + i / (TS::X * TS::Y);
            ok[j] = in_image(g, x, y, z);
            p[j] = ok[j] ? x + g.nx * (y + g.ny * z) : 0;
        }
#pragma unroll
        for (int j = 0; j < PER; ++j) l[j] = prev[p[j]];
#pragma unroll
        for (int j = 0; j < PER; ++j) l[j] = par[im.pix0 + l[j]] - im.pix0;
        int nroots = 0;
#pragma unroll
        for (int j = 0; j < PER; ++j)
            if (ok[j]) {
                cur[p[j]] = l[j];
                nroots += l[j] == p[j] ? 1 : 0;
            }
        int excl;
        int total = block_scan_excl(nroots, excl);
        if (threadIdx.x == 0) tile_cnt[t] = total;
    }
}

// out[b][k] = sum of the per-tile region counts of image b in layer k.
__global__ __launch_bounds__(NTHREADS) void k_img_counts(const Img *__restrict__ tab, Img one, int32_t nimg, int32_t nl,
                                                         int32_t ntiles_total, const int32_t *__restrict__ tile_cnt,
                                                         int64_t *const *__restrict__ outs, int64_t *one_out) {
    constexpr int U = 8;
    int b = blockIdx.x, k = blockIdx.y;
    if (b >= nimg || k >= nl) return;
    int32_t t0 = tab ? tab[b].tile0[TK_WF] : one.tile0[TK_WF];
    int32_t t1 = b + 1 < nimg ? tab[b + 1].tile0[TK_WF] : ntiles_total;
    const int32_t *c = tile_cnt + (size_t)k * ntiles_total;
    int s = 0;
    for (int32_t t = t0 + threadIdx.x; t < t1; t += NTHREADS * U) {
        int v[U];
#pragma unroll
        for (int j = 0; j < U; ++j) v[j] = t + j * NTHREADS < t1 ? c[t + j * NTHREADS] : 0;
#pragma unroll
        for (int j = 0; j < U; ++j) s += v[j];
    }
    int excl;
    int total = block_scan_excl(s, excl);
    int64_t *dst = tab ? outs[b] : one_out;
    if (threadIdx.x == 0 && dst) dst[k] = total;
}

// ---------------------------------------------------------------------------
template <int CONN, typename T, class Src>
static int launch_wf_edge_t(Launch &lc, const Src &src, const TileGrid &tg, int32_t layer, int32_t relabel,
                            const int32_t *par, uint64_t *key, int32_t *tile_cnt) {
    return lc.run("wf_edge", k_wf_edge<CONN, T, Src>, dim3(tg.grid), dim3(NTHREADS), src, tg.ntiles, layer, relabel,
                  par, key, tile_cnt);
}

template <class Src>
static int wf_edge_dispatch(Launch &lc, const Src &src, const TileGrid &tg, int conn, bool u16, int32_t layer,
                            int32_t relabel, const int32_t *par, uint64_t *key, int32_t *tile_cnt) {
    switch (conn) {
    case 4: return u16 ? launch_wf_edge_t<4, uint16_t>(lc, src, tg, layer, relabel, par, key, tile_cnt)
                       : launch_wf_edge_t<4, uint8_t>(lc, src, tg, layer, relabel, par, key, tile_cnt);
    case 8: return u16 ? launch_wf_edge_t<8, uint16_t>(lc, src, tg, layer, relabel, par, key, tile_cnt)
                       : launch_wf_edge_t<8, uint8_t>(lc, src, tg, layer, relabel, par, key, tile_cnt);
    case 6: return u16 ? launch_wf_edge_t<6, uint16_t>(lc, src, tg, layer, relabel, par, key, tile_cnt)
                       : launch_wf_edge_t<6, uint8_t>(lc, src, tg, layer, relabel, par, key, tile_cnt);
    case 26: return u16 ? launch_wf_edge_t<26, uint16_t>(lc, src, tg, layer, relabel, par, key, tile_cnt)
                        : launch_wf_edge_t<26, uint8_t>(lc, src, tg, layer, relabel, par, key, tile_cnt);
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

int compact_chunks(int32_t bound) { return (bound + CCHUNK - 1) / CCHUNK + 1; }

int wf_tiles(const Geom &g, int ndim) {
    if (ndim == 3)
        return ((g.nx + WfTile<3>::X - 1) / WfTile<3>::X) * ((g.ny + WfTile<3>::Y - 1) / WfTile<3>::Y) *
               ((g.nz + WfTile<3>::Z - 1) / WfTile<3>::Z);
    return ((g.nx + WfTile<2>::X - 1) / WfTile<2>::X) * ((g.ny + WfTile<2>::Y - 1) / WfTile<2>::Y) * g.nz;
}

template <class Src>
static int wf_init_impl(Launch &lc, const Src &src, const TileGrid &tg, int ndim, int32_t *list, int32_t *count,
                        uint64_t *key, int32_t *par, int32_t *tile_tmp, int32_t *tile_cnt0) {
    int rc = ndim == 3 ? lc.run("wf_init", k_root_count<3, Src>, dim3(tg.grid), dim3(NTHREADS), src, tg.ntiles,
                                tile_tmp, tile_cnt0)
                       : lc.run("wf_init", k_root_count<2, Src>, dim3(tg.grid), dim3(NTHREADS), src, tg.ntiles,
                                tile_tmp, tile_cnt0);
    if (rc) return rc;
    rc = lc.run("wf_init", k_scan, dim3(1), dim3(NTHREADS), tg.ntiles, (const int32_t *)nullptr, 1, tile_tmp, count);
    if (rc) return rc;
    return ndim == 3 ? lc.run("wf_init", k_root_write<3, Src>, dim3(tg.grid), dim3(NTHREADS), src, tg.ntiles,
                              (const int32_t *)tile_tmp, list, key, par)
                     : lc.run("wf_init", k_root_write<2, Src>, dim3(tg.grid), dim3(NTHREADS), src, tg.ntiles,
                              (const int32_t *)tile_tmp, list, key, par);
}

template <class Src>
static int wf_relabel_impl(Launch &lc, const Src &src, const TileGrid &tg, int ndim, int32_t layer, const int32_t *par,
                           int32_t *tile_cnt) {
    return ndim == 3 ? lc.run("wf_relabel", k_wf_relabel<3, Src>, dim3(tg.grid), dim3(NTHREADS), src, tg.ntiles, layer,
                              par, tile_cnt)
                     : lc.run("wf_relabel", k_wf_relabel<2, Src>, dim3(tg.grid), dim3(NTHREADS), src, tg.ntiles, layer,
                              par, tile_cnt);
}

#define WF_SRC_FUNCS(Src)                                                                                         \
    int launch_wf_init(Launch &lc, const Src &src, const TileGrid &tg, int ndim, int32_t *list, int32_t *count,  \
                       uint64_t *key, int32_t *par, int32_t *tile_tmp, int32_t *tile_cnt0) {                      \
        return wf_init_impl(lc, src, tg, ndim, list, count, key, par, tile_tmp, tile_cnt0);                       \
    }                                                                                                             \
    int launch_wf_edge(Launch &lc, const Src &src, const TileGrid &tg, int conn, bool u16, int32_t layer,        \
                       int32_t relabel, const int32_t *par, uint64_t *key, int32_t *tile_cnt) {                   \
        return wf_edge_dispatch(lc, src, tg, conn, u16, layer, relabel, par, key, tile_cnt);                     \
    }                                                                                                             \
    int launch_wf_relabel(Launch &lc, const Src &src, const TileGrid &tg, int ndim, int32_t layer,               \
                          const int32_t *par, int32_t *tile_cnt) {                                                \
        return wf_relabel_impl(lc, src, tg, ndim, layer, par, tile_cnt);                                          \
    }

WF_SRC_FUNCS(OneImg)
WF_SRC_FUNCS(ImgTable)

// Compaction of the survivors of a region list.
int launch_wf_compact(Launch &lc, int32_t bound, const int32_t *list_in, const int32_t *count_in, int32_t *list_out,
                      int32_t *count_out, const int32_t *par, uint64_t *key, int32_t *chunk_tmp) {
    int rc = lc.run("wf_compact", k_compact_count, chunk_grid(bound), dim3(NTHREADS), list_in, count_in, par, chunk_tmp);
    if (rc) return rc;
    rc = lc.run("wf_compact", k_scan, dim3(1), dim3(NTHREADS), 0, count_in, CCHUNK, chunk_tmp, count_out);
    if (rc) return rc;
    return lc.run("wf_compact", k_compact_write, chunk_grid(bound), dim3(NTHREADS), list_in, count_in, par,
                  (const int32_t *)chunk_tmp, list_out, key);
}

int launch_wf_union(Launch &lc, int32_t bound, const int32_t *list, const int32_t *count, uint64_t *key, int32_t *par) {
    return lc.run("wf_union", k_wf_union, list_grid(bound), dim3(NTHREADS), list, count, key, par);
}
int launch_wf_compress(Launch &lc, int32_t bound, const int32_t *list, const int32_t *count, int32_t *par) {
    return lc.run("wf_compress", k_wf_compress, list_grid(bound), dim3(NTHREADS), list, count, par);
}
int launch_img_counts(Launch &lc, const Img *tab, const Img &one, int32_t nimg, int32_t nl, int32_t ntiles_total,
                      const int32_t *tile_cnt, int64_t *const *outs, int64_t *one_out) {
    return lc.run("wf_counts", k_img_counts, dim3(nimg, nl), dim3(NTHREADS), tab, one, nimg, nl, ntiles_total, tile_cnt,
                  outs, one_out);
}

}  // namespace wsk
