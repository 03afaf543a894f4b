// waterfall.hip -- gfx950 kernels of the hierarchical waterfall (Section 4).
//
// Layer k joins every region R of layer k-1 with the region across its lowest
// boundary pass, key(R) = min over pixel pairs (p in R, q in N(p) outside R)
// of (max(I(p), I(q)), label(q)). Only the first layer looks at pixels; the
// later ones work on the region adjacency graph that pass leaves behind:
//
//   0. Region ids. Layer-0 regions (pixels carrying their own label) get dense
//      ids in pixel order, so id order is label order and every region table
//      is dense (rlist[id] = local label, par, key, mlab). The id of label l
//      is a rank: per 64 pixels one 16-byte record holds the root bitmap
//      word and the id of the first root at or after the word's first pixel,
//      so id(l) = base + popcount of the bits below l. These tables hold
//      0.25 byte per pixel, so the lookups stay in L2, unlike a pixel-indexed
//      table whose few live entries each cost a cache line.
//   1. Pixel pass, one workgroup per tile (it also writes every pixel's
//      region id, cimg, for step 4): every pixel pair (p, q), q in the
//      forward half of N(p), whose regions a != b differ is an edge
//      (a, b, max(I(p), I(q))). A tile's duplicates are merged in an LDS hash
//      (lowest height kept) and its edges go to the tile's slab. Each edge
//      lowers key[a] to (w, b) and key[b] to (w, a), first per region in LDS,
//      then with one 64-bit global atomicMin per (tile, region). Every pixel
//      pair lies in exactly one tile's forward half, so both directions of
//      all pairs are seen: the keys equal the definition above.
//   2. Union of every region with the target of its key (CAS hooking of the
//      larger id below the smaller, so a group's root is its smallest id =
//      smallest label), then compression: par[id] = root for every layer-0
//      id, and the layer's label of every layer-0 region, mlab[k][id].
//   3. Later layers, one workgroup per group of tiles: the slabs' edges are
//      mapped to the current roots, edges inside one region dropped,
//      duplicates merged, keys lowered as in 1; the survivors are written
//      back compacted at the group's start. Then 2 again.
//   4. One pass over the pixels writes every layer, out_k[p] =
//      mlab[k][cimg[p]], and counts each tile's pixels that carry their own
//      label (the regions of each layer).
//
// Hash tables that fill up fall back to direct global writes and atomics, so
// results never depend on table sizes. Images of a batch have their own
// chunks, hence disjoint id ranges, and edges only join pixels of one image.
#include "ws_device.h"
#include "ws_kernels.h"

namespace wsk {

constexpr uint64_t NOKEY = ~0ull;
constexpr uint64_t NOPAIR = ~0ull;

template <int NDIM> struct WfTile;
template <> struct WfTile<2> { static constexpr int X = 64, Y = 16, Z = 1; };
template <> struct WfTile<3> { static constexpr int X = 16, Y = 8, Z = 8; };
constexpr int WF_PIX = 1024;        // pixels per tile (both shapes)
constexpr int EBITS = 10;           // edge hash: 1024 slots
constexpr int ESLOTS = 1 << EBITS;
constexpr int MAXPROBE = 64;        // probes before a hash insert falls back
constexpr int RCH = 4096;           // pixels per region-id chunk (16 per thread)
constexpr int SCAN_B = NTHREADS * 16;  // elements per workgroup of the scans
constexpr int MAX_F = NTHREADS;     // tile groups merged per workgroup (one count per thread)
// Workgroup -> item runs per XCD (xcd_group): region ids and chunks that are
// close share table lines, so each XCD takes runs of 64 neighbouring items
// (measured best: fully contiguous ranges per XCD leave the 8 XCDs writing
// far-apart streams, runs of 1 re-fetch every table line into all 8 L2s).
constexpr int XG_OUT = 64;          // chunks per run in the output pass
// Ints per rank record of layers 2 .. nl-1 (whole 16-byte groups).
__host__ __device__ constexpr int layer_stride(int nl) { return nl < 3 ? 0 : (nl - 2 + 3) / 4 * 4; }
constexpr int XG_REG = 64;          // workgroups of 256 region ids per run

// Forward half of a neighbourhood: the neighbours with a larger linear index.
template <int CONN> __host__ __device__ constexpr bool forward(int k) { return nb_j<CONN>(k) > 13; }

// 1 if a forward neighbour can step back along x (axis 0) or y (axis 1): the
// diagonal neighbours of 8- and 26-connectivity. No forward neighbour steps
// back along z.
template <int CONN> __host__ __device__ constexpr int forward_back(int axis) {
    int r = 0;
    for (int k = 0; k < CONN; ++k)
        if (forward<CONN>(k) && (axis == 0 ? nb_dx<CONN>(k) : nb_dy<CONN>(k)) < 0) r = 1;
    return r;
}


// ---------------------------------------------------------------------------
// LDS hash tables. Inserts return false when MAXPROBE slots were taken by
// other keys; the caller then applies the update directly in global memory.
// ---------------------------------------------------------------------------
// Slot hashes from full-rate 24-bit multiplies (the ids' low bits vary most).
__device__ __forceinline__ uint32_t mix24(uint32_t a, uint32_t b) {
    uint32_t x = __umul24(a, 0x9E3779u) + __umul24(b, 0x45D9F3u);
    return x ^ (x >> 11);
}

__device__ __forceinline__ bool edge_insert(unsigned long long *ek, unsigned int *ew, uint64_t pair, uint32_t w) {
    uint32_t h = mix24((uint32_t)(pair >> 32), (uint32_t)pair) & (ESLOTS - 1);
    // Each probe is a single compare-and-swap (it writes only into an empty
    // slot): one LDS round trip whether the slot is empty or holds the pair.
    // Most inserts succeed at the first probe. The probe loop has a single
    // exit condition and stays rolled: a wave runs it whenever one of its
    // lanes missed, and its exec-mask bookkeeping is scalar work per
    // iteration (a loop with a separate found flag and break cost several
    // times more), while unrolled copies at every call site would spread the
    // hot code over far more instruction cache.
    unsigned long long cur = atomicCAS(&ek[h], (unsigned long long)NOPAIR, (unsigned long long)pair);
    bool miss = (cur != NOPAIR) & (cur != pair);  // one predicate, no short-circuit branches
    int probe = 1;
#pragma unroll 1
    while (miss & (probe < MAXPROBE)) {
        h = (h + 1) & (ESLOTS - 1);
        cur = atomicCAS(&ek[h], (unsigned long long)NOPAIR, (unsigned long long)pair);
        miss = (cur != NOPAIR) & (cur != pair);
        ++probe;
    }
    if (miss) return false;
    atomicMin(&ew[h], w);
    return true;
}

template <int BITS>
__device__ __forceinline__ bool region_insert(int *hk, unsigned long long *hv, int l, uint64_t v) {
    uint32_t h = mix24((uint32_t)l, (uint32_t)l >> 16) & ((1 << BITS) - 1);
    // probes as in edge_insert
    int cur = atomicCAS(&hk[h], -1, l);
    bool miss = (cur != -1) & (cur != l);
    int probe = 1;
#pragma unroll 1
    while (miss & (probe < MAXPROBE)) {
        h = (h + 1) & ((1 << BITS) - 1);
        cur = atomicCAS(&hk[h], -1, l);
        miss = (cur != -1) & (cur != l);
        ++probe;
    }
    if (miss) return false;
    atomicMin(&hv[h], (unsigned long long)v);
    return true;
}

// Both directions of edge (lo, hi, w) into the per-region minima.
template <int BITS>
__device__ __forceinline__ void edge_keys(int *hk, unsigned long long *hv, uint64_t *__restrict__ key, int32_t lo,
                                          int32_t hi, uint32_t w) {
    uint64_t vlo = ((uint64_t)w << 32) | (uint32_t)hi, vhi = ((uint64_t)w << 32) | (uint32_t)lo;
    if (!region_insert<BITS>(hk, hv, lo, vlo)) atomicMin((unsigned long long *)(key + lo), (unsigned long long)vlo);
    if (!region_insert<BITS>(hk, hv, hi, vhi)) atomicMin((unsigned long long *)(key + hi), (unsigned long long)vhi);
}

// An edge that found no hash slot: straight to the slab and the global keys.
__device__ __forceinline__ void edge_direct(int *ectr, uint64_t *__restrict__ key, uint64_t *__restrict__ ep,
                                            uint16_t *__restrict__ eww, size_t base, int32_t lo, int32_t hi,
                                            uint32_t w) {
    size_t pos = base + atomicAdd(ectr, 1);
    ep[pos] = ((uint64_t)(uint32_t)lo << 32) | (uint32_t)hi;
    eww[pos] = (uint16_t)w;
    atomicMin((unsigned long long *)(key + lo), (unsigned long long)(((uint64_t)w << 32) | (uint32_t)hi));
    atomicMin((unsigned long long *)(key + hi), (unsigned long long)(((uint64_t)w << 32) | (uint32_t)lo));
}

// Writes the edge hash's entries to the slab at base + ectr.., feeding their
// keys into the region hash. Wave-aggregated slot reservation.
template <int BITS>
__device__ __forceinline__ void emit_edges(const unsigned long long *ek, const unsigned int *ew, int *hk,
                                           unsigned long long *hv, int *ectr, uint64_t *__restrict__ key,
                                           uint64_t *__restrict__ ep, uint16_t *__restrict__ eww, size_t base) {
    for (int h0 = 0; h0 < ESLOTS; h0 += NTHREADS) {
        int h = h0 + threadIdx.x;
        unsigned long long pk = ek[h];
        bool v = pk != NOPAIR;
        uint64_t m = __ballot(v);
        if (m == 0) continue;  // wave-uniform
        int wbase = 0;
        if (__lane_id() == 0) wbase = atomicAdd(ectr, __popcll(m));
        wbase = __shfl(wbase, 0);
        if (!v) continue;
        size_t pos = base + wbase + __popcll(m & lanes_below());
        int32_t lo = (int32_t)(pk >> 32), hi = (int32_t)(uint32_t)pk;
        uint32_t w = ew[h];
        ep[pos] = (uint64_t)pk;
        eww[pos] = (uint16_t)w;
        edge_keys<BITS>(hk, hv, key, lo, hi, w);
    }
}

// Per-region minima of the LDS hash into the global keys.
template <int BITS>
__device__ __forceinline__ void flush_keys(const int *hk, const unsigned long long *hv, uint64_t *__restrict__ key) {
    for (int h = threadIdx.x; h < (1 << BITS); h += NTHREADS) {
        int l = hk[h];
        if (l >= 0) atomicMin((unsigned long long *)(key + l), hv[h]);
    }
}

// ---------------------------------------------------------------------------
// Scans. k_scan: one workgroup, exclusive scan of n counts in place, total to
// *total_out (n <= SCAN_B * 16 keeps it short). For longer arrays the counts
// are first summed per SCAN_B block (k_scan_part), the block sums scanned by
// k_scan, then every block rescanned with its offset (k_scan_apply).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(NTHREADS) void k_scan(int32_t n, int32_t *__restrict__ cnt, int32_t *__restrict__ total_out) {
    constexpr int U = 16;
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

__global__ __launch_bounds__(NTHREADS) void k_scan_part(int32_t n, const int32_t *__restrict__ cnt,
                                                        int32_t *__restrict__ part) {
    constexpr int U = SCAN_B / NTHREADS;
    int32_t b0 = blockIdx.x * SCAN_B;
    int32_t v[U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
        int32_t i = b0 + j * NTHREADS + threadIdx.x;
        v[j] = i < n ? cnt[i] : 0;
    }
    int s = 0;
#pragma unroll
    for (int j = 0; j < U; ++j) s += v[j];
    int excl;
    int total = block_scan_excl(s, excl);
    if (threadIdx.x == 0) part[blockIdx.x] = total;
}

__global__ __launch_bounds__(NTHREADS) void k_scan_apply(int32_t n, int32_t *__restrict__ cnt,
                                                         const int32_t *__restrict__ part) {
    constexpr int U = SCAN_B / NTHREADS;
    int32_t b0 = blockIdx.x * SCAN_B + threadIdx.x * U;  // a contiguous run per thread
    int32_t v[U];
#pragma unroll
    for (int j = 0; j < U; ++j) v[j] = b0 + j < n ? cnt[b0 + j] : 0;
    int s = 0;
#pragma unroll
    for (int j = 0; j < U; ++j) s += v[j];
    int excl;
    block_scan_excl(s, excl);
    int32_t run = part[blockIdx.x] + excl;
#pragma unroll
    for (int j = 0; j < U; ++j)
        if (b0 + j < n) {
            cnt[b0 + j] = run;
            run += v[j];
        }
}

// ---------------------------------------------------------------------------
// 0. Region ids. Chunk t covers pixels [lc*RCH, lc*RCH + RCH) of its image;
// element j of thread i is pixel lc*RCH + j*NTHREADS + i, so the ballot of
// wave w over element j is bitmap word j*NW + w of the chunk.
// ---------------------------------------------------------------------------
template <class Src>
__global__ __launch_bounds__(NTHREADS) void k_root_bits(Src src, int32_t nchunks, int32_t *__restrict__ ccnt,
                                                        RankWord *__restrict__ words) {
    constexpr int PER = RCH / NTHREADS;
    constexpr int NW = NTHREADS / 64;
    static_assert(PER * NW == 64, "one wave scans the chunk's words");
    __shared__ int wc[64];
    __shared__ unsigned long long wb[64];
    const int t = blockIdx.x;
    if (t >= nchunks) return;
    Img im;
    int lc;
    fetch(src, t, TK_CH, im, lc);
    const int32_t base = lc * RCH, end = im.g.n;
    const int lane = __lane_id(), w = threadIdx.x >> 6;
    int32_t l[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        int32_t p = base + j * NTHREADS + threadIdx.x;
        l[j] = p < end ? im.lab[p] : -1;
    }
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        uint64_t m = __ballot(l[j] == base + j * NTHREADS + (int)threadIdx.x);
        if (lane == 0) {
            wb[j * NW + w] = m;
            wc[j * NW + w] = __popcll(m);
        }
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        int v = wc[lane], x = v;
        for (int off = 1; off < 64; off <<= 1) {
            int y = __shfl_up(x, off);
            if (lane >= off) x += y;
        }
        RankWord rw;
        rw.bits = wb[lane];
        rw.base = x - v;  // in-chunk prefix; the chunk's first id is added after the scan
        rw.pad = 0;
        words[(size_t)t * 64 + lane] = rw;
        if (lane == 63) ccnt[t] = x;
    }
}

// Keys and parents of the nreg0 regions; chunk offsets into the rank words.
__global__ __launch_bounds__(NTHREADS) void k_wf_tables(const int32_t *__restrict__ nreg0, uint64_t *__restrict__ key,
                                                        int32_t *__restrict__ par, int32_t nwords,
                                                        RankWord *__restrict__ words, const int32_t *__restrict__ coff) {
    const int32_t n = *nreg0;
    for (int32_t c = blockIdx.x * NTHREADS + threadIdx.x; c < n; c += gridDim.x * NTHREADS) {
        key[c] = NOKEY;
        par[c] = c;
    }
    for (int32_t i = blockIdx.x * NTHREADS + threadIdx.x; i < nwords; i += gridDim.x * NTHREADS)
        words[i].base += coff[i >> 6];
}

// ---------------------------------------------------------------------------
// 1. Pixel pass of layer 0 (keys of layer 1 and the tiles' edge slabs; the
// region id of every own pixel into cimg, the labels of the own roots into
// rlist). Labels are clamped to the image
// and ids to [0, nreg0) so that labels that are not canonical cannot address
// outside the tables.
// ---------------------------------------------------------------------------
template <int CONN, typename T, class Src>
__global__ __launch_bounds__(NTHREADS) void k_wf_pix(Src src, int32_t ntiles, const RankWord *__restrict__ words,
                                                     const int32_t *__restrict__ nreg0, int32_t *__restrict__ cimg,
                                                     int32_t *__restrict__ rlist, uint64_t *__restrict__ key,
                                                     uint64_t *__restrict__ ep, uint16_t *__restrict__ eww,
                                                     int32_t *__restrict__ ecnt, int32_t cap) {
    constexpr int NDIM = ndim_of<CONN>();
    using TS = WfTile<NDIM>;
    // Only forward pairs are formed, so the staged box extends one cell past
    // the tile on the high side of every axis and one cell below it only along
    // the axes where a forward neighbour steps back.
    constexpr int LX = forward_back<CONN>(0), LY = forward_back<CONN>(1);
    constexpr int SX = TS::X + LX + 1, SY = TS::Y + LY + 1, SZ = NDIM == 3 ? TS::Z + 1 : 1;
    constexpr int CELLS = SX * SY * SZ;
    constexpr int PIX = TS::X * TS::Y * TS::Z;
    static_assert(PIX == WF_PIX && PIX % NTHREADS == 0, "whole waves per tile");
    // sL/sI hold the tile's ids and grey values; once the edges are collected
    // the same words hold the region hash (keys, then 64-bit minima)
    constexpr int RBITS = 9;
    // ids int32 + grey T per cell (5 or 6 B: the arrays and hashes of 2D
    // tiles and of uint8 volumes stay within the 20 KB of eight workgroups
    // per CU; uint16 volumes run seven)
    constexpr int CBYTES = CELLS * (4 + (int)sizeof(T)), HBYTES = (1 << RBITS) * 12;
    constexpr int SBUF = ((CBYTES > HBYTES ? CBYTES : HBYTES) + 7) / 8;
    static_assert((NDIM == 3 && sizeof(T) == 2) || SBUF * 8 + ESLOTS * 12 + 16 <= 20480, "eight workgroups per CU");
    __shared__ unsigned long long sbuf[SBUF];
    __shared__ unsigned long long ek[ESLOTS];
    __shared__ unsigned int ew[ESLOTS];
    __shared__ int ectr;
    int *sL = (int *)sbuf;
    T *sI = (T *)(sL + CELLS);
    int *hk = (int *)sbuf;
    unsigned long long *hv = sbuf + (1 << RBITS) / 2;
    if ((int)blockIdx.x >= ntiles) return;
    const int t = xcd_tile(blockIdx.x, ntiles);
    Img im;
    int lt;
    fetch(src, t, TK_WF, im, lt);
    const Geom &g = im.g;
    const T *I = (const T *)im.grey;
    const int32_t *L0 = im.lab;
    int ox, oy, oz;
    tile_xyz<TS::X, TS::Y, TS::Z>(g, lt, ox, oy, oz);
    const int32_t nr = *nreg0;
    const uint32_t cmax = nr > 0 ? (uint32_t)(nr - 1) : 0u;
    {
        constexpr int PER = (CELLS + NTHREADS - 1) / NTHREADS;
        int32_t idx[PER], lv[PER];
        T gv[PER];
        bool ok[PER], own[PER];
        uint64_t ownm;
        const uint64_t okm = box_cells<SX, SY, SZ, PER, LX, LY, TS::X, TS::Y, TS::Z>(
            g, ox - LX, oy - LY, oz,
            [&](int j, int32_t i) {
                idx[j] = i;
                lv[j] = L0[i];
                gv[j] = I[i];
            },
            &ownm);
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            ok[j] = okm >> j & 1;
            own[j] = ownm >> j & 1;
        }
        // region ids by rank, one record load per cell
        const size_t w0 = (size_t)im.tile0[TK_CH] * 64;
        RankWord rw[PER];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            int32_t l = (uint32_t)lv[j] < (uint32_t)g.n ? lv[j] : 0;
            rw[j] = words[w0 + (l >> 6)];
        }
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            int c = threadIdx.x + j * NTHREADS;
            uint64_t below = (1ull << (lv[j] & 63)) - 1ull;
            uint32_t cv = (uint32_t)(rw[j].base + __popcll(rw[j].bits & below));
            cv = cv <= cmax ? cv : cmax;
            if (c < CELLS) {
                sL[c] = ok[j] ? (int)cv : -1;
                sI[c] = ok[j] ? gv[j] : (T)0;
            }
            if (own[j]) {
                cimg[(size_t)im.pix0 + idx[j]] = (int32_t)cv;
                if (lv[j] == idx[j]) rlist[cv] = idx[j];
            }
        }
    }
    for (int h = threadIdx.x; h < ESLOTS; h += NTHREADS) {
        ek[h] = NOPAIR;
        ew[h] = 0xffffffffu;
    }
    if (threadIdx.x == 0) ectr = 0;
    __syncthreads();
    const size_t base = (size_t)t * (size_t)cap;
    for (int i = threadIdx.x; i < PIX; i += NTHREADS) {  // uniform trip count
        int x = i % TS::X, y = (i / TS::X) % TS::Y, z = i / (TS::X * TS::Y);
        int s = (z * SY + (y + LY)) * SX + (x + LX);
        const int a = sL[s];
        const uint32_t v = (uint32_t)sI[s];
        // every forward neighbour's id and grey value is read before any
        // test (one LDS wait, no branch per neighbour)
        int nbL[CONN];
        uint32_t nbI[CONN];
#pragma unroll
        for (int k = 0; k < CONN; ++k) {
            if (!forward<CONN>(k)) continue;
            const int o = s + nb_dx<CONN>(k) + SX * (nb_dy<CONN>(k) + SY * nb_dz<CONN>(k));
            nbL[k] = sL[o];
            nbI[k] = (uint32_t)sI[o];
        }
        if (a < 0) continue;
#pragma unroll
        for (int k = 0; k < CONN; ++k) {
            if (!forward<CONN>(k)) continue;
            const int b = nbL[k];
            if (b < 0 || b == a) continue;
            const uint32_t wq = nbI[k];
            const uint32_t w = v > wq ? v : wq;
            int32_t lo = a < b ? a : b, hi = a < b ? b : a;
            uint64_t pair = ((uint64_t)(uint32_t)lo << 32) | (uint32_t)hi;
            if (!edge_insert(ek, ew, pair, w)) edge_direct(&ectr, key, ep, eww, base, lo, hi, w);
        }
    }
    __syncthreads();
    for (int h = threadIdx.x; h < (1 << RBITS); h += NTHREADS) {
        hk[h] = -1;
        hv[h] = NOKEY;
    }
    __syncthreads();
    emit_edges<RBITS>(ek, ew, hk, hv, &ectr, key, ep, eww, base);
    __syncthreads();
    flush_keys<RBITS>(hk, hv, key);
    if (threadIdx.x == 0) ecnt[t] = ectr;
}

// ---------------------------------------------------------------------------
// 3. Edge pass of a later layer. Workgroup g merges the f groups of gin tiles
// starting at tile g*gin*f (their edges sit at the start of each group's
// slab range, counts at ecnt[first tile of the group]) into one group of
// gin*f tiles. par maps every layer-0 id to its current root.
//
// In-place safety: outputs are written at increasing offsets from the merged
// group's start, never more of them than inputs consumed so far, and input e
// (in concatenated order) lies at an offset >= e because every group holds at
// most its capacity; a barrier after each batch's loads ends its reads first.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(NTHREADS) void k_wf_level(int32_t ntiles, int32_t gin, int32_t f, int32_t cap,
                                                       const int32_t *__restrict__ par, uint64_t *__restrict__ key,
                                                       uint64_t *__restrict__ ep, uint16_t *__restrict__ eww,
                                                       int32_t *__restrict__ ecnt) {
    constexpr int RBITS = 9;  // 512 region slots: with 1024 edge slots the pass fits eight workgroups per CU
    __shared__ unsigned long long ek[ESLOTS];
    __shared__ unsigned int ew[ESLOTS];
    __shared__ int hk[1 << RBITS];
    __shared__ unsigned long long hv[1 << RBITS];
    __shared__ int soff[MAX_F];
    __shared__ int stotal, ectr;
    const int32_t t0 = blockIdx.x * gin * f;
    if (t0 >= ntiles) return;
    const int32_t nsub = min(f, (ntiles - t0 + gin - 1) / gin);
    {
        int c = (int)threadIdx.x < nsub ? ecnt[t0 + threadIdx.x * gin] : 0;
        int excl;
        int total = block_scan_excl(c, excl);
        soff[threadIdx.x] = excl;
        if (threadIdx.x == 0) {
            stotal = total;
            ectr = 0;
        }
    }
    for (int h = threadIdx.x; h < ESLOTS; h += NTHREADS) {
        ek[h] = NOPAIR;
        ew[h] = 0xffffffffu;
    }
    for (int h = threadIdx.x; h < (1 << RBITS); h += NTHREADS) {
        hk[h] = -1;
        hv[h] = NOKEY;
    }
    __syncthreads();
    const int32_t total = stotal;
    const size_t base = (size_t)t0 * (size_t)cap;
    // Up to four subgroups (the merge factor the host uses): an edge's
    // subgroup is the number of later subgroup starts at or below it (the
    // offsets are non-decreasing), from three offsets read once, without a
    // search loop per edge
    const bool few = f <= 4;
    int o1 = 0x7fffffff, o2 = 0x7fffffff, o3 = 0x7fffffff;
    if (few) {
        if (nsub > 1) o1 = soff[1];
        if (nsub > 2) o2 = soff[2];
        if (nsub > 3) o3 = soff[3];
    }
    // LEV_U edges per thread per batch: all their loads, then all their parent
    // gathers, are issued before the first wait (two round trips per batch)
    constexpr int LEV_U = 8;
    for (int32_t e0 = 0; e0 < total; e0 += NTHREADS * LEV_U) {  // uniform trip count
        int32_t ra[LEV_U], rb[LEV_U];
        uint32_t w[LEV_U];
        size_t at[LEV_U];
#pragma unroll
        for (int u = 0; u < LEV_U; ++u) {
            int32_t e = e0 + u * NTHREADS + (int)threadIdx.x;
            at[u] = 0;
            if (e < total) {
                if (few) {
                    const int lo = (o1 <= e ? 1 : 0) + (o2 <= e ? 1 : 0) + (o3 <= e ? 1 : 0);
                    const int so = lo == 0 ? 0 : lo == 1 ? o1 : lo == 2 ? o2 : o3;  // soff[0] == 0
                    at[u] = (size_t)(t0 + lo * gin) * (size_t)cap + (size_t)(e - so);
                } else {
                    int lo = 0, hi = nsub - 1;
                    while (lo < hi) {
                        int mid = (lo + hi + 1) >> 1;
                        if (soff[mid] <= e) lo = mid;
                        else hi = mid - 1;
                    }
                    at[u] = (size_t)(t0 + lo * gin) * (size_t)cap + (size_t)(e - soff[lo]);
                }
            }
        }
        // branch-free: lanes past the end read slab entry 0 (allocated, any
        // contents) and parent 0, and use neither
        uint64_t pr[LEV_U];
#pragma unroll
        for (int u = 0; u < LEV_U; ++u) {
            pr[u] = ep[at[u]];
            w[u] = (uint32_t)eww[at[u]];
        }
#pragma unroll
        for (int u = 0; u < LEV_U; ++u) {
            const bool ok = e0 + u * NTHREADS + (int)threadIdx.x < total;
            ra[u] = par[ok ? (int32_t)(pr[u] >> 32) : 0];
            rb[u] = par[ok ? (int32_t)(uint32_t)pr[u] : 0];
        }
        // this batch's reads precede every write below: a workgroup's vector
        // memory operations pass through its CU's cache in issue order, so a
        // store issued after the barrier cannot overtake a load issued before it
        __syncthreads();
#pragma unroll
        for (int u = 0; u < LEV_U; ++u) {
            int32_t e = e0 + u * NTHREADS + (int)threadIdx.x;
            if (e < total && ra[u] != rb[u]) {
                int32_t lo = ra[u] < rb[u] ? ra[u] : rb[u], hi = ra[u] < rb[u] ? rb[u] : ra[u];
                uint64_t pair = ((uint64_t)(uint32_t)lo << 32) | (uint32_t)hi;
                if (!edge_insert(ek, ew, pair, w[u])) edge_direct(&ectr, key, ep, eww, base, lo, hi, w[u]);
            }
        }
    }
    __syncthreads();
    emit_edges<RBITS>(ek, ew, hk, hv, &ectr, key, ep, eww, base);
    __syncthreads();
    flush_keys<RBITS>(hk, hv, key);
    if (threadIdx.x == 0) ecnt[t0] = ectr;
}

// ---------------------------------------------------------------------------
// 2. Union of every live region with the target of its key, in two kernels so
// that most hooks are plain stores (device atomics execute at the memory side
// and cost far more): first every region whose target has a smaller id hooks
// to it -- only the region itself writes its parent, and it is a root, so no
// other write can race -- then the regions whose target has a larger id are
// united by CAS hooking, which finds most of them already joined. Parents
// keep pointing to smaller ids, so every root is its tree's smallest id.
// Keys are reset to NOKEY as they are consumed; only roots ever get new ones.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(NTHREADS) void k_wf_hook(const int32_t *__restrict__ nreg0,
                                                      const uint64_t *__restrict__ key, int32_t *__restrict__ par) {
    const int32_t n = *nreg0;
    for (int32_t c = xcd_group(blockIdx.x, gridDim.x, XG_REG) * NTHREADS + threadIdx.x; c < n;
         c += gridDim.x * NTHREADS) {
        uint64_t kk = key[c];
        int32_t tg = (int32_t)(uint32_t)(kk & 0xffffffffull);
        if (kk != NOKEY && tg < c) par[c] = tg;
    }
}

__global__ __launch_bounds__(NTHREADS) void k_wf_union(const int32_t *__restrict__ nreg0, uint64_t *__restrict__ key,
                                                       int32_t *__restrict__ par) {
    const int32_t n = *nreg0;
    for (int32_t c = xcd_group(blockIdx.x, gridDim.x, XG_REG) * NTHREADS + threadIdx.x; c < n;
         c += gridDim.x * NTHREADS) {
        uint64_t kk = key[c];
        if (kk == NOKEY) continue;
        key[c] = NOKEY;
        int32_t tg = (int32_t)(uint32_t)(kk & 0xffffffffull);
        if (tg > c) gunion_halve(par, c, tg);
    }
}

__global__ __launch_bounds__(NTHREADS) void k_wf_compress(const int32_t *__restrict__ nreg0, int32_t *__restrict__ par,
                                                          const int32_t *__restrict__ rlist,
                                                          int32_t *__restrict__ mlab_k) {
    const int32_t n = *nreg0;
    for (int32_t c = xcd_group(blockIdx.x, gridDim.x, XG_REG) * NTHREADS + threadIdx.x; c < n;
         c += gridDim.x * NTHREADS) {
        int32_t r = gfind_ro(par, c);
        par[c] = r;
        mlab_k[c] = rlist[r];
    }
}

// ---------------------------------------------------------------------------
// 2b. Layers >= 2 over the roots of layer 1 only. After layer 1's union the
// regions that are still roots (par[c] == c) are listed in increasing id
// order, R1[i], with their rank in id1[r]; layer 1's compression then gives
// every region c the rank of its layer-1 root, id1[c]. Keys and parent
// changes of later layers only ever concern such roots, so their union and
// compression walk R1 (a fraction of the regions), and their label tables are
// indexed by rank: M_k[i] = label of R1[i] in layer k.
// ---------------------------------------------------------------------------
// Roots among c in [0, nreg0) per SCAN_B block of ids (a run of 16 ids per thread).
__device__ __forceinline__ uint32_t root_mask16(const int32_t *__restrict__ par, int32_t c0, int32_t n) {
    uint32_t m = 0;
    if (c0 + 16 <= n) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int4 v = *(const int4 *)(par + c0 + 4 * q);
            m |= (v.x == c0 + 4 * q ? 1u : 0u) << (4 * q);
            m |= (v.y == c0 + 4 * q + 1 ? 1u : 0u) << (4 * q + 1);
            m |= (v.z == c0 + 4 * q + 2 ? 1u : 0u) << (4 * q + 2);
            m |= (v.w == c0 + 4 * q + 3 ? 1u : 0u) << (4 * q + 3);
        }
    } else {
        for (int j = 0; j < 16; ++j)
            if (c0 + j < n && par[c0 + j] == c0 + j) m |= 1u << j;
    }
    return m;
}

__global__ __launch_bounds__(NTHREADS) void k_root_count(const int32_t *__restrict__ nreg0,
                                                         const int32_t *__restrict__ par, int32_t *__restrict__ bcnt) {
    static_assert(SCAN_B == NTHREADS * 16, "16 ids per thread");
    const int32_t n = *nreg0;
    if ((int64_t)blockIdx.x * SCAN_B >= n) {
        if (threadIdx.x == 0) bcnt[blockIdx.x] = 0;
        return;
    }
    const int32_t c0 = blockIdx.x * SCAN_B + threadIdx.x * 16;
    int excl;
    const int total = block_scan_excl(__popc(root_mask16(par, c0, n)), excl);
    if (threadIdx.x == 0) bcnt[blockIdx.x] = total;
}

// R1[rank] = root and id1[root * ids] = rank, from the scanned block counts. The
// list holds at most `cap` roots (a layer at least halves the regions of every
// image, so valid labels never reach it); ranks past it are clamped.
__global__ __launch_bounds__(NTHREADS) void k_root_scatter(const int32_t *__restrict__ nreg0,
                                                           const int32_t *__restrict__ par,
                                                           const int32_t *__restrict__ bcnt, int32_t *__restrict__ R1,
                                                           int32_t *__restrict__ id1, int32_t ids, int32_t cap) {
    const int32_t n = *nreg0;
    if ((int64_t)blockIdx.x * SCAN_B >= n) return;
    const int32_t c0 = blockIdx.x * SCAN_B + threadIdx.x * 16;
    const uint32_t m = root_mask16(par, c0, n);
    int excl;
    block_scan_excl(__popc(m), excl);
    int32_t rank = bcnt[blockIdx.x] + excl;
    for (uint32_t b = m; b; b &= b - 1) {
        const int32_t c = c0 + __ffs(b) - 1;
        if (rank < cap) R1[rank] = c;
        id1[(size_t)c * ids] = rank < cap ? rank : cap - 1;
        ++rank;
    }
}

// Layer 1's compression, also giving every region the rank of its root:
// region c's layer-1 label at mlab1[c * ms], that rank at id1[c * ms] (the
// two interleave in one record per region).
__global__ __launch_bounds__(NTHREADS) void k_wf_compress1(const int32_t *__restrict__ nreg0, int32_t *__restrict__ par,
                                                           const int32_t *__restrict__ rlist,
                                                           int32_t *__restrict__ mlab1, int32_t *__restrict__ id1,
                                                           int32_t ms) {
    const int32_t n = *nreg0;
    for (int32_t c = xcd_group(blockIdx.x, gridDim.x, XG_REG) * NTHREADS + threadIdx.x; c < n;
         c += gridDim.x * NTHREADS) {
        int32_t r = gfind_ro(par, c);
        par[c] = r;
        if (ms == 2 && id1 == mlab1 + 1) {
            // one 8-byte store of the region's record (the root's rank was
            // set by the root list; its record's rank is rewritten unchanged)
            ((int2 *)mlab1)[c] = make_int2(rlist[r], id1[(size_t)r * 2]);
        } else {
            mlab1[(size_t)c * ms] = rlist[r];
            if (r != c) id1[(size_t)c * ms] = id1[(size_t)r * ms];  // roots already hold their rank
        }
    }
}

__global__ __launch_bounds__(NTHREADS) void k_wf_hook_l(const int32_t *__restrict__ n1p, int32_t cap,
                                                        const int32_t *__restrict__ R1,
                                                        const uint64_t *__restrict__ key, int32_t *__restrict__ par) {
    const int32_t n = min(*n1p, cap);
    for (int32_t i = xcd_group(blockIdx.x, gridDim.x, XG_REG) * NTHREADS + threadIdx.x; i < n;
         i += gridDim.x * NTHREADS) {
        const int32_t c = R1[i];
        uint64_t kk = key[c];
        int32_t tg = (int32_t)(uint32_t)(kk & 0xffffffffull);
        if (kk != NOKEY && tg < c) par[c] = tg;
    }
}

__global__ __launch_bounds__(NTHREADS) void k_wf_union_l(const int32_t *__restrict__ n1p, int32_t cap,
                                                         const int32_t *__restrict__ R1,
                                                         uint64_t *__restrict__ key, int32_t *__restrict__ par) {
    const int32_t n = min(*n1p, cap);
    for (int32_t i = xcd_group(blockIdx.x, gridDim.x, XG_REG) * NTHREADS + threadIdx.x; i < n;
         i += gridDim.x * NTHREADS) {
        const int32_t c = R1[i];
        uint64_t kk = key[c];
        if (kk == NOKEY) continue;
        key[c] = NOKEY;
        int32_t tg = (int32_t)(uint32_t)(kk & 0xffffffffull);
        if (tg > c) gunion_halve(par, c, tg);
    }
}

__global__ __launch_bounds__(NTHREADS) void k_wf_compress_l(const int32_t *__restrict__ n1p, int32_t cap,
                                                            const int32_t *__restrict__ R1, int32_t *__restrict__ par,
                                                            const int32_t *__restrict__ rlist,
                                                            int32_t *__restrict__ Mk, int32_t ls) {
    const int32_t n = min(*n1p, cap);
    for (int32_t i = xcd_group(blockIdx.x, gridDim.x, XG_REG) * NTHREADS + threadIdx.x; i < n;
         i += gridDim.x * NTHREADS) {
        const int32_t c = R1[i];
        int32_t r = gfind_ro(par, c);
        par[c] = r;
        Mk[(size_t)i * ls] = rlist[r];
    }
}

// ---------------------------------------------------------------------------
// 4. Layers 1 .. nl-1 of every pixel from its region id, chunk by chunk. The
// label tables: for nl == 2 layer 1 by region id at mlab; for nl >= 3 one
// record {layer-1 label, rank of the layer-1 root} per region id at mlab
// (mstride records), then the root list (hstride ints), then per rank one
// record of layers 2 .. nl-1 (layer_stride(nl) ints, a multiple of 4).
// (RCH consecutive pixels of one image), and per chunk the number of pixels
// carrying their own label in each layer, cnt[k * nchunks + t]. Layer 0's
// count is the chunk's root count, the difference of consecutive chunk
// offsets. A thread owns runs of 4 consecutive pixels: 16-byte loads and
// stores when the image's layers are 16-byte aligned, else scalar accesses.
// With nl == 1 only layer 0 is counted. Layers are written one after the
// other, each as one contiguous span per chunk. This form serves any nl;
// k_wf_out_p below serves 2 <= nl <= 8.
// ---------------------------------------------------------------------------
template <class Src>
__global__ __launch_bounds__(NTHREADS) void k_wf_out(Src src_ch, int32_t nchunks, int32_t nl,
                                                     const int32_t *__restrict__ cimg,
                                                     const int32_t *__restrict__ nreg0,
                                                     const int32_t *__restrict__ coff,
                                                     const int32_t *__restrict__ mlab, int64_t mstride,
                                                     int64_t hstride, int32_t *__restrict__ cnt) {
    constexpr int RUNS = RCH / (4 * NTHREADS);  // runs of 4 pixels per thread
    static_assert(RUNS * 4 * NTHREADS == RCH, "whole runs per chunk");
    __shared__ int kc;
    if ((int)blockIdx.x >= nchunks) return;
    const int t = xcd_group(blockIdx.x, nchunks, XG_OUT);
    Img im;
    int lc;
    fetch(src_ch, t, TK_CH, im, lc);
    const int32_t nr = *nreg0;
    if (threadIdx.x == 0) cnt[t] = (t + 1 < nchunks ? coff[t + 1] : nr) - coff[t];
    if (nl == 1) return;
    const Geom &g = im.g;
    const int32_t base = lc * RCH, n = g.n;
    const int32_t *ci = cimg + im.pix0;
    const bool vec = ((im.pix0 | n) & 3) == 0 && ((uintptr_t)im.lab & 15) == 0;
    const uint32_t cmax = nr > 0 ? (uint32_t)(nr - 1) : 0u;
    int32_t c[RUNS][4];
    int32_t p0[RUNS];
#pragma unroll
    for (int r = 0; r < RUNS; ++r) {
        p0[r] = base + (r * NTHREADS + (int)threadIdx.x) * 4;
        if (vec && p0[r] + 3 < n) {
            int4 q = *(const int4 *)(ci + p0[r]);
            c[r][0] = q.x;
            c[r][1] = q.y;
            c[r][2] = q.z;
            c[r][3] = q.w;
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) c[r][e] = p0[r] + e < n ? ci[p0[r] + e] : 0;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) c[r][e] = (uint32_t)c[r][e] <= cmax ? c[r][e] : (int32_t)cmax;
    }
    // nl >= 3: one record per region id {layer-1 label, rank of the layer-1
    // root}, then per rank a record of the layers 2 .. nl-1 (lstride ints)
    const int lstride = layer_stride(nl);
    int32_t rk[RUNS][4];  // rank of the layer-1 root (tables of layers >= 2)
    if (nl >= 3) {
#pragma unroll
        for (int r = 0; r < RUNS; ++r)
#pragma unroll
            for (int e = 0; e < 4; ++e) rk[r][e] = mlab[2 * (size_t)c[r][e] + 1];
    }
    const int32_t *lay = mlab + 2 * (size_t)mstride + (size_t)hstride;
#pragma unroll 1
    for (int k = 1; k < nl; ++k) {
        int32_t *out = im.lab + (size_t)k * (size_t)n;
        if (threadIdx.x == 0) kc = 0;
        __syncthreads();
        int own = 0;
#pragma unroll
        for (int r = 0; r < RUNS; ++r) {
            int32_t v[4];
#pragma unroll
            for (int e = 0; e < 4; ++e)
                v[e] = k == 1 ? mlab[(nl >= 3 ? 2 : 1) * (size_t)c[r][e]]
                              : lay[(size_t)rk[r][e] * lstride + (k - 2)];
#pragma unroll
            for (int e = 0; e < 4; ++e) own += (p0[r] + e < n && v[e] == p0[r] + e) ? 1 : 0;
            if (vec && p0[r] + 3 < n) {
                *(int4 *)(out + p0[r]) = make_int4(v[0], v[1], v[2], v[3]);
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (p0[r] + e < n) out[p0[r] + e] = v[e];
            }
        }
        for (int off = 32; off > 0; off >>= 1) own += __shfl_xor(own, off);
        if (__lane_id() == 0 && own) atomicAdd(&kc, own);
        __syncthreads();
        if (threadIdx.x == 0) cnt[(size_t)k * nchunks + t] = kc;
    }
}

// The same pass for NLM = nl - 1 <= 7 layers above layer 0. Loads and stores
// of a wave complete through one in-order counter, so a wave that waits for a
// gather also waits for every store it issued before it. Each thread
// therefore gathers everything first (layer 1 and the rank of the layer-1
// root by region id, then layers 2 .. NLM by that rank) and only then stores:
// one wave's stores drain while other waves gather. 512 threads per chunk
// keep that at 8 pixels (two runs of 4) per thread. A pixel whose region id
// equals the previous pixel's in its run gathers nothing and copies that
// pixel's values, so a gather instruction carries fewer active lanes (the
// address unit, not HBM, bounds these gathers). Own-label counts are wave
// ballots summed into one LDS counter per layer, with one barrier per chunk.
constexpr int WF_OUT_MAXNL = 8;
constexpr int OUT_T = 512;
constexpr int OUT_RUNS = RCH / (4 * OUT_T);

// Table gathers as raw buffer loads: a 32-bit byte offset per pixel against a
// per-table descriptor (base, size), so no 64-bit per-lane address is formed.
// Offsets past the table's size read 0.
constexpr int BUF_CONFIG = 0x00020000;  // raw 32-bit buffer, gfx9 family
__device__ __forceinline__ __amdgpu_buffer_rsrc_t table_rsrc(const int32_t *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, (int)bytes, BUF_CONFIG);
}
// Pixels with bit 4r + e of `need` gather; the others copy their run's
// previous pixel in wf_fill, once the loads are back.
__device__ __forceinline__ void wf_gather(int32_t (&v)[OUT_RUNS][4], const uint32_t (&off)[OUT_RUNS][4],
                                          __amdgpu_buffer_rsrc_t rs, uint32_t need) {
#pragma unroll
    for (int r = 0; r < OUT_RUNS; ++r)
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (need >> (4 * r + e) & 1u) v[r][e] = __builtin_amdgcn_raw_buffer_load_b32(rs, (int)off[r][e], 0, 0);
}
__device__ __forceinline__ void wf_fill(int32_t (&v)[OUT_RUNS][4], uint32_t need) {
#pragma unroll
    for (int r = 0; r < OUT_RUNS; ++r)
#pragma unroll
        for (int e = 1; e < 4; ++e)
            if (!(need >> (4 * r + e) & 1u)) v[r][e] = v[r][e - 1];
}

typedef int wf_v4i __attribute__((ext_vector_type(4)));
__device__ __forceinline__ int wf_emit(const int32_t (&v)[OUT_RUNS][4], const int32_t (&p0)[OUT_RUNS], int32_t n,
                                       bool vec, int32_t *__restrict__ out) {
    int own = 0;
    // 16-byte runs as raw buffer stores (32-bit offsets against the layer's
    // descriptor); a layer of n < 2^30 pixels stays below 4 GiB
    const __amdgpu_buffer_rsrc_t rs = table_rsrc(out, (uint32_t)((size_t)n * 4));
#pragma unroll
    for (int r = 0; r < OUT_RUNS; ++r) {
#pragma unroll
        for (int e = 0; e < 4; ++e) own += __popcll(__ballot(p0[r] + e < n && v[r][e] == p0[r] + e));
        if (vec && p0[r] + 3 < n) {
            wf_v4i d = {v[r][0], v[r][1], v[r][2], v[r][3]};
            __builtin_amdgcn_raw_buffer_store_b128(d, rs, p0[r] * 4, 0, 0);
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (p0[r] + e < n) out[p0[r] + e] = v[r][e];
        }
    }
    return own;
}

// Table bases: t[0] layer 1 by region id (nl == 2, gathered as raw buffer
// loads) or the 8-byte region records (nl >= 3); t[1] the 16-byte rank
// records of layers 2 .. nl-1. Records cut the gathers of a pixel from nl to
// 1 + ceil((nl - 2) / 4), each to one cache line.
struct WfTabs {
    const int32_t *t[2];
    uint32_t bytes;    // size of t[0] when nl == 2 (< 4 GiB: larger arenas take the layer-by-layer kernel)
};

template <class Src, int NLM>
__global__ __launch_bounds__(OUT_T) void k_wf_out_p(Src src_ch, int32_t nchunks, const int32_t *__restrict__ cimg,
                                                    const int32_t *__restrict__ nreg0,
                                                    const int32_t *__restrict__ coff, WfTabs tabs,
                                                    int32_t *__restrict__ cnt) {
    static_assert(OUT_RUNS * 4 * OUT_T == RCH, "whole runs per chunk");
    __shared__ int kc[WF_OUT_MAXNL];
    if ((int)blockIdx.x >= nchunks) return;
    const int t = xcd_group(blockIdx.x, nchunks, XG_OUT);
    Img im;
    int lc;
    fetch(src_ch, t, TK_CH, im, lc);
    const int32_t nr = *nreg0;
    if (threadIdx.x == 0) cnt[t] = (t + 1 < nchunks ? coff[t + 1] : nr) - coff[t];
    if ((int)threadIdx.x < WF_OUT_MAXNL) kc[threadIdx.x] = 0;
    __syncthreads();
    const int32_t base = lc * RCH, n = im.g.n;
    const int32_t *ci = cimg + im.pix0;
    const bool vec = ((im.pix0 | n) & 3) == 0 && ((uintptr_t)im.lab & 15) == 0;
    const uint32_t cmax = nr > 0 ? (uint32_t)(nr - 1) : 0u;
    uint32_t off[OUT_RUNS][4];
    int32_t p0[OUT_RUNS];
    uint32_t need = 0;
#pragma unroll
    for (int r = 0; r < OUT_RUNS; ++r) {
        p0[r] = base + (r * OUT_T + (int)threadIdx.x) * 4;
        int32_t c[4];
        if (vec && p0[r] + 3 < n) {
            int4 q = *(const int4 *)(ci + p0[r]);
            c[0] = q.x;
            c[1] = q.y;
            c[2] = q.z;
            c[3] = q.w;
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) c[e] = p0[r] + e < n ? ci[p0[r] + e] : 0;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            off[r][e] = ((uint32_t)c[e] <= cmax ? (uint32_t)c[e] : cmax) * 4u;
            if (e == 0 || off[r][e] != off[r][e - 1]) need |= 1u << (4 * r + e);
        }
    }
    int32_t V[NLM][OUT_RUNS][4];
    uint32_t need_r = need;
    if constexpr (NLM == 1) {
        wf_gather(V[0], off, table_rsrc(tabs.t[0], tabs.bytes), need);  // layer 1, by region id
    } else {
        // one 8-byte record per region id: {layer-1 label, rank of the
        // layer-1 root}; then, by that rank, 16-byte records of four later
        // layers each (once per change of the rank along the run: layer-1
        // regions are larger, so its runs are longer than the region id's)
        const int2 *T1 = (const int2 *)tabs.t[0];
        const int4 *TL = (const int4 *)tabs.t[1];
        constexpr int G = (NLM - 1 + 3) / 4;  // 16-byte groups per rank record
        int32_t rk[OUT_RUNS][4];
#pragma unroll
        for (int r = 0; r < OUT_RUNS; ++r)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (need >> (4 * r + e) & 1u) {
                    const int2 q = T1[off[r][e] >> 2];
                    V[0][r][e] = q.x;
                    rk[r][e] = q.y;
                }
        wf_fill(rk, need);
        need_r = 0;
#pragma unroll
        for (int r = 0; r < OUT_RUNS; ++r)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (e == 0 || rk[r][e] != rk[r][e - 1]) need_r |= 1u << (4 * r + e);
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
            for (int r = 0; r < OUT_RUNS; ++r)
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (need_r >> (4 * r + e) & 1u) {
                        const int4 q = TL[(size_t)(uint32_t)rk[r][e] * G + g];
                        if (1 + 4 * g < NLM) V[1 + 4 * g][r][e] = q.x;
                        if (2 + 4 * g < NLM) V[2 + 4 * g][r][e] = q.y;
                        if (3 + 4 * g < NLM) V[3 + 4 * g][r][e] = q.z;
                        if (4 + 4 * g < NLM) V[4 + 4 * g][r][e] = q.w;
                    }
    }
    int own[NLM];
#pragma unroll
    for (int k = 1; k <= NLM; ++k) {
        wf_fill(V[k - 1], k == 1 ? need : need_r);
        own[k - 1] = wf_emit(V[k - 1], p0, n, vec, im.lab + (size_t)k * (size_t)n);
    }
    if (__lane_id() == 0) {
#pragma unroll
        for (int k = 0; k < NLM; ++k)
            if (own[k]) atomicAdd(&kc[k + 1], own[k]);
    }
    __syncthreads();
    if ((int)threadIdx.x >= 1 && (int)threadIdx.x <= NLM) cnt[(size_t)threadIdx.x * nchunks + t] = kc[threadIdx.x];
}

template <class Src>
static int wf_out_pipelined(Launch &lc, const Src &src_ch, int32_t nchunks, int32_t nl, const int32_t *cimg,
                            const int32_t *nreg0, const int32_t *coff, const int32_t *mlab, int64_t mstride,
                            int64_t hstride, int32_t *cnt) {
    dim3 grid(nchunks > 0 ? nchunks : 1);
    WfTabs tabs{};
    tabs.bytes = (uint32_t)((size_t)mstride * 4);
    tabs.t[0] = mlab;
    if (nl >= 3) tabs.t[1] = mlab + 2 * (size_t)mstride + (size_t)hstride;
    switch (nl - 1) {
#define WF_OUT_P(M)                                                                                               \
    case M:                                                                                                       \
        return lc.run("wf_out", k_wf_out_p<Src, M>, grid, dim3(OUT_T), src_ch, nchunks, cimg, nreg0, coff, tabs,    \
                      cnt);
        WF_OUT_P(1)
        WF_OUT_P(2)
        WF_OUT_P(3)
        WF_OUT_P(4)
        WF_OUT_P(5)
        WF_OUT_P(6)
        WF_OUT_P(7)
#undef WF_OUT_P
        default:
            return -1;
    }
}

// out[b][k] = sum of the per-chunk region counts of image b in layer k.
__global__ __launch_bounds__(NTHREADS) void k_img_counts(const Img *__restrict__ tab, Img one, int32_t nimg, int32_t nl,
                                                         int32_t ntiles_total, const int32_t *__restrict__ tile_cnt,
                                                         int64_t *const *__restrict__ outs, int64_t *one_out) {
    constexpr int U = 8;
    int b = blockIdx.x, k = blockIdx.y;
    if (b >= nimg || k >= nl) return;
    int32_t t0 = tab ? tab[b].tile0[TK_CH] : one.tile0[TK_CH];
    int32_t t1 = b + 1 < nimg ? tab[b + 1].tile0[TK_CH] : ntiles_total;
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

static inline dim3 list_grid(int32_t n) {
    int32_t b = (n + NTHREADS - 1) / NTHREADS;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    return dim3(b);
}

// ---------------------------------------------------------------------------
// Reconstruction waterfall (Alg. 4 Steps V-VI before each re-run of the
// watershed, Alg. 5). The raised image is kept as uint16.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(NTHREADS) void k_grey_u16(const T *__restrict__ in, uint16_t *__restrict__ out, int32_t n) {
    for (int32_t p = blockIdx.x * NTHREADS + threadIdx.x; p < n; p += gridDim.x * NTHREADS) out[p] = (uint16_t)in[p];
}

// Step VI: I(p) = max(I(p), newmin(region of p)), where newmin is the height
// part of the region's key (Step V's lowest boundary pass) and M = 65535 for
// a region without boundary.
__global__ __launch_bounds__(NTHREADS) void k_recon_raise(uint16_t *__restrict__ I, const int32_t *__restrict__ cimg,
                                                          const uint64_t *__restrict__ key,
                                                          const int32_t *__restrict__ nreg0, int32_t n) {
    const int32_t nr = *nreg0;
    const uint32_t cmax = nr > 0 ? (uint32_t)(nr - 1) : 0u;
    for (int32_t p = blockIdx.x * NTHREADS + threadIdx.x; p < n; p += gridDim.x * NTHREADS) {
        uint32_t c = (uint32_t)cimg[p];
        c = c <= cmax ? c : cmax;
        uint64_t kk = key[c];
        uint32_t m = kk == NOKEY ? 65535u : (uint32_t)(kk >> 32);
        if (I[p] < m) I[p] = (uint16_t)m;
    }
}

int launch_grey_u16(Launch &lc, const void *in, bool u16, uint16_t *out, int32_t n) {
    dim3 grid = list_grid(n);
    return u16 ? lc.run("recon", k_grey_u16<uint16_t>, grid, dim3(NTHREADS), (const uint16_t *)in, out, n)
               : lc.run("recon", k_grey_u16<uint8_t>, grid, dim3(NTHREADS), (const uint8_t *)in, out, n);
}
int launch_recon_raise(Launch &lc, uint16_t *I, const int32_t *cimg, const uint64_t *key, const int32_t *nreg0,
                       int32_t n) {
    return lc.run("recon", k_recon_raise, list_grid(n), dim3(NTHREADS), I, cimg, key, nreg0, n);
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

int wf_tiles(const Geom &g, int ndim) {
    if (ndim == 3)
        return ((g.nx + WfTile<3>::X - 1) / WfTile<3>::X) * ((g.ny + WfTile<3>::Y - 1) / WfTile<3>::Y) *
               ((g.nz + WfTile<3>::Z - 1) / WfTile<3>::Z);
    return ((g.nx + WfTile<2>::X - 1) / WfTile<2>::X) * ((g.ny + WfTile<2>::Y - 1) / WfTile<2>::Y) * g.nz;
}
int wf_chunks(int32_t n) { return (n + RCH - 1) / RCH; }
int wf_slab_cap(int conn) { return conn / 2 * WF_PIX; }
int wf_max_merge() { return MAX_F; }
int scan_tmp_len(int32_t n) { return n <= SCAN_B * 16 ? 1 : (n + SCAN_B - 1) / SCAN_B + 1; }

// Exclusive scan of n ints in place, total to *total_out; tmp holds
// scan_tmp_len(n) ints.
int launch_scan(Launch &lc, int32_t n, int32_t *data, int32_t *tmp, int32_t *total_out) {
    if (n <= SCAN_B * 16) return lc.run("wf_ids", k_scan, dim3(1), dim3(NTHREADS), n, data, total_out);
    int32_t nb = (n + SCAN_B - 1) / SCAN_B;
    int rc = lc.run("wf_ids", k_scan_part, dim3(nb), dim3(NTHREADS), n, (const int32_t *)data, tmp);
    if (rc) return rc;
    if ((rc = lc.run("wf_ids", k_scan, dim3(1), dim3(NTHREADS), nb, tmp, total_out))) return rc;
    return lc.run("wf_ids", k_scan_apply, dim3(nb), dim3(NTHREADS), n, data, (const int32_t *)tmp);
}

int launch_wf_level(Launch &lc, int32_t ntiles, int32_t gin, int32_t f, const int32_t *par, uint64_t *key,
                    const EdgeSlabs &es) {
    if (f < 1 || f > MAX_F || gin < 1) return -1;
    int64_t gout = (int64_t)gin * f;
    int64_t ng = ((int64_t)ntiles + gout - 1) / gout;
    return lc.run("wf_level", k_wf_level, dim3((uint32_t)(ng > 0 ? ng : 1)), dim3(NTHREADS), ntiles, gin, f, es.cap,
                  par, key, es.p, es.w, es.cnt);
}

int launch_root_list(Launch &lc, int32_t bound, const int32_t *nreg0, const int32_t *par, int32_t *R1, int32_t *id1,
                     int32_t ids, int32_t cap, int32_t *scratch, int32_t *n1) {
    const int32_t nb = (bound + SCAN_B - 1) / SCAN_B > 0 ? (bound + SCAN_B - 1) / SCAN_B : 1;
    int32_t *bcnt = scratch, *tmp = scratch + nb;
    int rc = lc.run("wf_union", k_root_count, dim3(nb), dim3(NTHREADS), nreg0, par, bcnt);
    if (rc) return rc;
    if ((rc = launch_scan(lc, nb, bcnt, tmp, n1))) return rc;
    return lc.run("wf_union", k_root_scatter, dim3(nb), dim3(NTHREADS), nreg0, par, (const int32_t *)bcnt, R1, id1,
                  ids, cap);
}
int root_list_tmp_len(int32_t bound) {
    const int32_t nb = (bound + SCAN_B - 1) / SCAN_B > 0 ? (bound + SCAN_B - 1) / SCAN_B : 1;
    return nb + scan_tmp_len(nb);
}
int launch_wf_compress1(Launch &lc, int32_t bound, const int32_t *nreg0, int32_t *par, const int32_t *rlist,
                        int32_t *mlab1, int32_t *id1, int32_t ms) {
    return lc.run("wf_compress", k_wf_compress1, list_grid(bound), dim3(NTHREADS), nreg0, par, rlist, mlab1, id1, ms);
}
// The root list holds a few per cent of the pixels on natural images: its
// grids are sized for bound / 32 ids (grid-stride loops cover any length), so
// later layers do not dispatch thousands of empty workgroups.
static inline dim3 root_grid(int32_t bound) { return list_grid(bound / 32 > 0 ? bound / 32 : 1); }
int launch_wf_union_l(Launch &lc, int32_t bound, const int32_t *n1, int32_t cap, const int32_t *R1, uint64_t *key,
                      int32_t *par) {
    int rc = lc.run("wf_union", k_wf_hook_l, root_grid(bound), dim3(NTHREADS), n1, cap, R1, (const uint64_t *)key,
                    par);
    if (rc) return rc;
    return lc.run("wf_union", k_wf_union_l, root_grid(bound), dim3(NTHREADS), n1, cap, R1, key, par);
}
int launch_wf_compress_l(Launch &lc, int32_t bound, const int32_t *n1, int32_t cap, const int32_t *R1, int32_t *par,
                         const int32_t *rlist, int32_t *Mk, int32_t ls) {
    return lc.run("wf_compress", k_wf_compress_l, root_grid(bound), dim3(NTHREADS), n1, cap, R1, par, rlist, Mk, ls);
}
int launch_wf_union(Launch &lc, int32_t bound, const int32_t *nreg0, uint64_t *key, int32_t *par) {
    int rc = lc.run("wf_union", k_wf_hook, list_grid(bound), dim3(NTHREADS), nreg0, (const uint64_t *)key, par);
    if (rc) return rc;
    return lc.run("wf_union", k_wf_union, list_grid(bound), dim3(NTHREADS), nreg0, key, par);
}
int launch_wf_compress(Launch &lc, int32_t bound, const int32_t *nreg0, int32_t *par, const int32_t *rlist,
                       int32_t *mlab_k) {
    return lc.run("wf_compress", k_wf_compress, list_grid(bound), dim3(NTHREADS), nreg0, par, rlist, mlab_k);
}
int launch_img_counts(Launch &lc, const Img *tab, const Img &one, int32_t nimg, int32_t nl, int32_t ntiles_total,
                      const int32_t *tile_cnt, int64_t *const *outs, int64_t *one_out) {
    return lc.run("wf_counts", k_img_counts, dim3(nimg, nl), dim3(NTHREADS), tab, one, nimg, nl, ntiles_total, tile_cnt,
                  outs, one_out);
}

template <class Src>
static int wf_ids_impl(Launch &lc, const Src &src_ch, int32_t nchunks, int32_t bound, const WfIds &ids,
                       int32_t *scan_tmp, int32_t *nreg0, uint64_t *key, int32_t *par) {
    dim3 grid(nchunks > 0 ? nchunks : 1);
    int rc = lc.run("wf_ids", k_root_bits<Src>, grid, dim3(NTHREADS), src_ch, nchunks, ids.coff, ids.words);
    if (rc) return rc;
    if ((rc = launch_scan(lc, nchunks, ids.coff, scan_tmp, nreg0))) return rc;
    if (!key) return 0;  // region counts only
    int32_t nwords = nchunks * 64;
    return lc.run("wf_ids", k_wf_tables, list_grid(bound > nwords ? bound : nwords), dim3(NTHREADS),
                  (const int32_t *)nreg0, key, par, nwords, ids.words, (const int32_t *)ids.coff);
}

template <int CONN, typename T, class Src>
static int wf_pix_t(Launch &lc, const Src &src, const TileGrid &tg, const WfIds &ids, const int32_t *nreg0,
                    int32_t *cimg, int32_t *rlist, uint64_t *key, const EdgeSlabs &es) {
    if (es.cap < wf_slab_cap(CONN)) return -1;  // a tile's forward pairs must fit its slab
    return lc.run("wf_pix", k_wf_pix<CONN, T, Src>, dim3(tg.grid), dim3(NTHREADS), src, tg.ntiles,
                  (const RankWord *)ids.words, nreg0, cimg, rlist, key, es.p, es.w, es.cnt, es.cap);
}

template <class Src>
static int wf_pix_dispatch(Launch &lc, const Src &src, const TileGrid &tg, int conn, bool u16, const WfIds &ids,
                           const int32_t *nreg0, int32_t *cimg, int32_t *rlist, uint64_t *key, const EdgeSlabs &es) {
#define WF_PIX_ARGS lc, src, tg, ids, nreg0, cimg, rlist, key, es
    switch (conn) {
    case 4: return u16 ? wf_pix_t<4, uint16_t>(WF_PIX_ARGS) : wf_pix_t<4, uint8_t>(WF_PIX_ARGS);
    case 8: return u16 ? wf_pix_t<8, uint16_t>(WF_PIX_ARGS) : wf_pix_t<8, uint8_t>(WF_PIX_ARGS);
    case 6: return u16 ? wf_pix_t<6, uint16_t>(WF_PIX_ARGS) : wf_pix_t<6, uint8_t>(WF_PIX_ARGS);
    case 26: return u16 ? wf_pix_t<26, uint16_t>(WF_PIX_ARGS) : wf_pix_t<26, uint8_t>(WF_PIX_ARGS);
    default: return -1;
    }
#undef WF_PIX_ARGS
}

#define WF_SRC_FUNCS(Src)                                                                                          \
    int launch_wf_ids(Launch &lc, const Src &src_ch, int32_t nchunks, int32_t bound, const WfIds &ids,            \
                      int32_t *scan_tmp, int32_t *nreg0, uint64_t *key, int32_t *par) {                           \
        return wf_ids_impl(lc, src_ch, nchunks, bound, ids, scan_tmp, nreg0, key, par);                           \
    }                                                                                                              \
    int launch_wf_pix(Launch &lc, const Src &src, const TileGrid &tg, int conn, bool u16, const WfIds &ids,       \
                      const int32_t *nreg0, int32_t *cimg, int32_t *rlist, uint64_t *key, const EdgeSlabs &es) {  \
        return wf_pix_dispatch(lc, src, tg, conn, u16, ids, nreg0, cimg, rlist, key, es);                         \
    }                                                                                                              \
    int launch_wf_out(Launch &lc, const Src &src_ch, int32_t nchunks, int32_t nl, const int32_t *cimg,            \
                      const int32_t *nreg0, const int32_t *coff, const int32_t *mlab, int64_t mstride,           \
                      int64_t hstride, int32_t *cnt) {                                                            \
        if (nl >= 2 && nl <= WF_OUT_MAXNL && (size_t)mstride * 4 <= 0xffffffffu)                                 \
            return wf_out_pipelined<Src>(lc, src_ch, nchunks, nl, cimg, nreg0, coff, mlab, mstride, hstride,     \
                                         cnt);                                                                    \
        return lc.run("wf_out", k_wf_out<Src>, dim3(nchunks > 0 ? nchunks : 1), dim3(NTHREADS), src_ch, nchunks, \
                      nl, cimg, nreg0, coff, mlab, mstride, hstride, cnt);                                        \
    }

WF_SRC_FUNCS(OneImg)
WF_SRC_FUNCS(ImgTable)

}  // namespace wsk
