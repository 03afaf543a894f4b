// ws_device.h -- device-side helpers shared by the gfx950 kernels of libws.
//
// Pixel order: p = x + nx*(y + ny*z) (row-major order required by Step I of
// Alg. 1). Neighbourhoods are enumerated in increasing linear index, which for
// in-image pixels is the lexicographic order of (dz, dy, dx).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wsk {

constexpr int32_t INF = 0x7fffffff;   // unresolved plateau distance
constexpr int32_t SENT = 0x10000;     // grey value of out-of-image cells (> any uint16)
constexpr int NTHREADS = 256;          // threads of every tile kernel (4 waves of 64)

// Unsigned division by a runtime constant for dividends below 2^31
// (multiply-high with a rounded-up magic number, shift s = ceil(log2 d)).
struct FastDiv {
    uint32_t d = 1, m = 1, s = 0;
    FastDiv() = default;
    explicit FastDiv(uint32_t div) : d(div) {
        s = 0;
        while ((1ull << s) < div) ++s;
        m = (uint32_t)((((1ull << 32) * ((1ull << s) - div)) / div) + 1);
    }
    __device__ __forceinline__ uint32_t div(uint32_t n) const { return (__umulhi(n, m) + n) >> s; }
};

// Image geometry passed by value to every kernel.
struct Geom {
    int32_t nx, ny, nz, n;     // sizes, n = nx*ny*nz < 2^31
    int32_t ntx, nty, ntz;     // tile grid
    FastDiv dnx, dny;          // division by nx and ny
};

// One image of a call. A single-image call passes one Img by value; a batched
// call passes a device table of them plus, per tiling, a tile -> image map.
// Scratch that spans the whole call (distances, region keys and parents) is
// addressed with pix0 + local pixel index ("arena" index).
enum TileKind { TK_WS = 0, TK_WF = 1, TK_GR = 2, TK_CH = 3 };  // TK_CH: waterfall region-id chunks

struct Img {
    Geom g;               // sizes (the ntx/nty/ntz fields hold the watershed tiling)
    int32_t pix0;         // arena offset of the image's pixel 0
    int32_t tile0[4];     // first tile of the image in each tiling (global tile index)
    int32_t slot0;        // first partial-maximum word (gradient)
    const void *grey;     // quantised gradient (u8/u16)
    int32_t *lab;         // label layers: layer k at lab + k * g.n
    const float *fimg;    // gradient input
    void *gout;           // gradient output
    float *mag;           // gradient magnitude
};

struct OneImg {
    Img im;
};
struct ImgTable {
    const Img *tab;       // device table of images
    const int32_t *map;   // global tile -> image, for the kernel's tiling
};

__device__ __forceinline__ void fetch(const OneImg &s, int t, int, Img &im, int &lt) {
    im = s.im;
    lt = t;
}
__device__ __forceinline__ void fetch(const ImgTable &s, int t, int kind, Img &im, int &lt) {
    int b = s.map[t];
    im = s.tab[b];
    lt = t - im.tile0[kind];
}

// Workgroups of a launch are dispatched to the chip's XCDs round-robin
// (workgroup b to XCD b % NXCD). xcd_tile maps workgroup b to tile t so that
// every XCD works through one contiguous range of tiles: neighbouring tiles,
// whose halos share cache lines, then meet in the same L2. A bijection on
// [0, n).
constexpr int NXCD = 8;
__device__ __forceinline__ int xcd_tile(int b, int n) {
    int q = n / NXCD, r = n % NXCD, x = b % NXCD, s = b / NXCD;
    return x * q + (x < r ? x : r) + s;
}

// Like xcd_tile, but every XCD takes runs of G consecutive items in turn, so
// that the XCDs together sweep one front of 8 G items through [0, n) while
// each reuses the cache lines its own run shares. Items past the last whole
// front map to themselves. A bijection on [0, n).
__device__ __forceinline__ int xcd_group(int b, int n, int G) {
    if (G < 1) G = 1;
    const int F = NXCD * G, full = n / F * F;
    if (b >= full) return b;
    const int w = b % F;
    return b - w + (w % NXCD) * G + w / NXCD;
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

__device__ __forceinline__ uint64_t lanes_below() { return (1ull << __lane_id()) - 1ull; }

// Origin of local tile lt of a tiling with tile shape (X, Y, Z).
template <int X, int Y, int Z>
__device__ __forceinline__ void tile_xyz(const Geom &g, int lt, int &ox, int &oy, int &oz) {
    int ntx = (g.nx + X - 1) / X, nty = (g.ny + Y - 1) / Y;
    int tx = lt % ntx, r = lt / ntx;
    ox = tx * X;
    oy = (r % nty) * Y;
    oz = (r / nty) * Z;
}

// Neighbour k of a connectivity, as an index j into the 3x3x3 cube
// (j = 9*(dz+1) + 3*(dy+1) + (dx+1)); increasing k gives increasing j, hence
// increasing linear pixel index.
template <int CONN>
__host__ __device__ constexpr int nb_j(int k) {
    return CONN == 4 ? 10 + 2 * k
         : CONN == 8 ? (k < 4 ? 9 + k : 10 + k)
         : CONN == 6 ? (k == 0 ? 4 : (k == 5 ? 22 : 10 + 2 * (k - 1)))
         : (k < 13 ? k : k + 1);
}
template <int CONN> __host__ __device__ constexpr int nb_dx(int k) { return nb_j<CONN>(k) % 3 - 1; }
template <int CONN> __host__ __device__ constexpr int nb_dy(int k) { return (nb_j<CONN>(k) / 3) % 3 - 1; }
template <int CONN> __host__ __device__ constexpr int nb_dz(int k) { return nb_j<CONN>(k) / 9 - 1; }
template <int CONN> __host__ __device__ constexpr int ndim_of() { return (CONN == 4 || CONN == 8) ? 2 : 3; }

// Watershed tile shapes (pixels per workgroup), by shape id: the id's last
// decimal digit is the dimensionality (2 and 3 are the defaults). LPER is the
// number of plateau-list entries per thread in Step II (tiles with more
// unresolved plateau pixels relax every pixel instead).
template <int SH> struct TileShape;
template <> struct TileShape<2> { static constexpr int X = 64, Y = 32, Z = 1, LPER = 1; };
template <> struct TileShape<12> { static constexpr int X = 128, Y = 16, Z = 1, LPER = 1; };
template <> struct TileShape<22> { static constexpr int X = 32, Y = 32, Z = 1, LPER = 1; };
template <> struct TileShape<32> { static constexpr int X = 64, Y = 64, Z = 1, LPER = 2; };
template <> struct TileShape<3> { static constexpr int X = 32, Y = 8, Z = 8, LPER = 1; };
template <> struct TileShape<13> { static constexpr int X = 16, Y = 16, Z = 8, LPER = 1; };
template <> struct TileShape<23> { static constexpr int X = 32, Y = 16, Z = 8, LPER = 2; };
template <> struct TileShape<33> { static constexpr int X = 16, Y = 16, Z = 16, LPER = 2; };
template <int SH> __host__ __device__ constexpr int shape_ndim() { return SH % 10; }

// The same table for host code: the sizes of shape `sh`, false for an
// unknown id.
inline bool tile_dims(int sh, int &X, int &Y, int &Z) {
    switch (sh) {
#define WS_TILE_CASE(S)     \
    case S:                 \
        X = TileShape<S>::X; \
        Y = TileShape<S>::Y; \
        Z = TileShape<S>::Z; \
        return true;
        WS_TILE_CASE(2) WS_TILE_CASE(12) WS_TILE_CASE(22) WS_TILE_CASE(32)
        WS_TILE_CASE(3) WS_TILE_CASE(13) WS_TILE_CASE(23) WS_TILE_CASE(33)
#undef WS_TILE_CASE
    default:
        return false;
    }
}

// LDS layout of a tile of shape SH with a ring of width R.
template <int SH, int R>
struct Lds {
    using T = TileShape<SH>;
    static constexpr int SX = T::X + 2 * R;
    static constexpr int SY = T::Y + 2 * R;
    static constexpr int SZ = shape_ndim<SH>() == 3 ? T::Z + 2 * R : 1;
    static constexpr int RZ = shape_ndim<SH>() == 3 ? R : 0;
    static constexpr int CELLS = SX * SY * SZ;
    __device__ static constexpr int at(int x, int y, int z) { return ((z + RZ) * SY + (y + R)) * SX + (x + R); }
    template <int CONN> __device__ static constexpr int off(int k) {
        return nb_dx<CONN>(k) + SX * (nb_dy<CONN>(k) + SY * nb_dz<CONN>(k));
    }
};

__device__ __forceinline__ void pixel_coords(const Geom &g, int32_t p, int &x, int &y, int &z) {
    uint32_t q1 = g.dnx.div((uint32_t)p);
    x = p - (int32_t)q1 * g.nx;
    uint32_t q2 = g.dny.div(q1);
    y = (int32_t)q1 - (int32_t)q2 * g.ny;
    z = (int32_t)q2;
}

__device__ __forceinline__ bool in_image(const Geom &g, int x, int y, int z) {
    return x >= 0 && x < g.nx && y >= 0 && y < g.ny && z >= 0 && z < g.nz;
}

// Walks this thread's cells of a box of SX x SY x SZ cells whose first cell
// sits at image coordinates (bx, by, bz); the thread's cell j is
// c = threadIdx.x + j * NTHREADS in x-fastest order. For every j it calls
// load(j, index) with the cell's image index (0 for cells outside the box or
// the image), so loads are issued as soon as their address is known, and
// returns a mask with bit j set for cells inside both the box and the
// image. With a core (KX x KY x KZ cells from box cell (KX0, KY0, 0)), *core
// gets the same bits for the cells inside it. Cell coordinates advance by
// constant mixed-radix steps instead of a division per cell, and a box
// inside the image (most tiles) skips the per-cell bounds tests (the test is
// uniform over the workgroup).
template <bool INNER, int SX, int SY, int SZ, int PER, int KX0, int KY0, int KX, int KY, int KZ, class Load>
__device__ __forceinline__ uint64_t box_walk(const Geom &g, int bx, int by, int bz, Load &load, uint64_t &km) {
    constexpr int CELLS = SX * SY * SZ;
    static_assert(PER * NTHREADS >= CELLS && (PER - 1) * NTHREADS < CELLS && PER <= 64, "cells per thread");
    constexpr int SR = NTHREADS % SX, SB = (NTHREADS / SX) % SY, SA = NTHREADS / (SX * SY);
    const int t = threadIdx.x;
    int cx = t % SX, cy = (t / SX) % SY, cz = t / (SX * SY);
    uint64_t okm = 0;
    km = 0;
    const int32_t base = bx + g.nx * (by + g.ny * bz);
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const bool live = j < PER - 1 || t + j * NTHREADS < CELLS;
        bool ok;
        int32_t i;
        if (INNER) {
            ok = live;
            i = ok ? base + cx + g.nx * (cy + g.ny * cz) : 0;
        } else {
            const int x = bx + cx, y = by + cy, z = bz + cz;
            ok = live && x >= 0 && x < g.nx && y >= 0 && y < g.ny && z >= 0 && z < g.nz;
            i = ok ? x + g.nx * (y + g.ny * z) : 0;
        }
        load(j, i);
        okm |= (uint64_t)(ok ? 1 : 0) << j;
        if (KX > 0)
            km |= (uint64_t)(ok && cx >= KX0 && cx < KX0 + KX && cy >= KY0 && cy < KY0 + KY && cz < KZ ? 1 : 0) << j;
        cx += SR;
        const int c1 = cx >= SX ? 1 : 0;
        cx -= c1 * SX;
        cy += SB + c1;
        const int c2 = cy >= SY ? 1 : 0;
        cy -= c2 * SY;
        cz += SA + c2;
    }
    return okm;
}

template <int SX, int SY, int SZ, int PER, int KX0 = 0, int KY0 = 0, int KX = 0, int KY = 0, int KZ = 0, class Load>
__device__ __forceinline__ uint64_t box_cells(const Geom &g, int bx, int by, int bz, Load &&load,
                                              uint64_t *core = nullptr) {
    uint64_t km;
    const uint64_t okm =
        (bx >= 0 && by >= 0 && bz >= 0 && bx + SX <= g.nx && by + SY <= g.ny && bz + SZ <= g.nz)
            ? box_walk<true, SX, SY, SZ, PER, KX0, KY0, KX, KY, KZ>(g, bx, by, bz, load, km)
            : box_walk<false, SX, SY, SZ, PER, KX0, KY0, KX, KY, KZ>(g, bx, by, bz, load, km);
    if (core) *core = km;
    return okm;
}

// Batched, branch-free load of a box of cells (SX x SY x SZ, first cell at
// image coordinates (bx, by, bz)) into LDS: every thread first computes all its
// addresses (cells outside the image read pixel 0 and are replaced by `fill`),
// then issues all its loads back to back, then writes LDS, so a workgroup
// waits for one memory latency instead of one per cell. (The initial Step II
// pass stages its two-cell ring this way: with box_cells' two code paths its
// 21 to 32 cells per thread measured slower.)
template <int SX, int SY, int SZ, typename T, typename V>
__device__ __forceinline__ void load_box(const Geom &g, int bx, int by, int bz, const T *__restrict__ src, V *dst,
                                         V fill) {
    constexpr int CELLS = SX * SY * SZ;
    constexpr int PER = (CELLS + NTHREADS - 1) / NTHREADS;
    int32_t idx[PER];
    bool ok[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        int c = threadIdx.x + j * NTHREADS;
        int cx = c % SX, cy = (c / SX) % SY, cz = c / (SX * SY);
        int x = bx + cx, y = by + cy, z = bz + cz;
        ok[j] = c < CELLS && x >= 0 && x < g.nx && y >= 0 && y < g.ny && z >= 0 && z < g.nz;
        idx[j] = ok[j] ? x + g.nx * (y + g.ny * z) : 0;
    }
    T v[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) v[j] = src[idx[j]];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        int c = threadIdx.x + j * NTHREADS;
        if (c < CELLS) dst[c] = ok[j] ? (V)v[j] : fill;
    }
}

// Parent loads and stores of the global union-find go through the caches
// (wavefront-scope relaxed atomics compile to plain loads and stores): a
// stale parent is still an ancestor, because parents only ever move to an
// ancestor, and the one update that must be seen device-wide, hooking a root,
// is a device-scope CAS that fails and returns the current parent when the
// root was hooked meanwhile.
__device__ __forceinline__ int32_t ld_par(const int32_t *a) {
    return __hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// Union-find over a parent array in global memory with parent[x] <= x:
// roots are self loops, and a union always hooks the larger root below the
// smaller one, so a tree's root is the smallest index in it. Every chase
// moves to strictly smaller indices, so finds end even on stale parents, and
// every failed CAS returns a smaller parent, so unions end too.
//
// Root of x without writing: safe while other threads store final roots into
// the same array (a path-halving write could replace a final root by an
// intermediate ancestor).
__device__ __forceinline__ int32_t gfind_ro(const int32_t *par, int32_t x) {
    for (;;) {
        int32_t px = ld_par(par + x);
        if (px == x) return x;
        x = px;
    }
}

// Root of x, splitting the path on the way: every visited node's parent
// moves to its grandparent (a plain store; it only ever moves a parent to an
// ancestor). A grandparent equal to the parent ends the walk at once (the
// parent is a root), one load earlier than re-reading it.
__device__ __forceinline__ int32_t gfind(int32_t *par, int32_t x) {
    for (;;) {
        int32_t px = ld_par(par + x);
        if (px == x) return x;
        int32_t ppx = ld_par(par + px);
        if (ppx == px) return px;
        __hip_atomic_store(par + x, ppx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        x = px;
    }
}

// Union of the trees of a and b: one find after the other (the watershed's
// crossings, whose paths are one to three steps long).
__device__ __forceinline__ void gunion(int32_t *par, int32_t a, int32_t b) {
    a = gfind(par, a);
    b = gfind(par, b);
    while (a != b) {
        if (a < b) { int32_t t = a; a = b; b = t; }
        int32_t old = atomicCAS(par + a, a, b);
        if (old == a) return;
        a = gfind(par, old);
        b = gfind(par, b);
    }
}

// Union of the trees of a and b with both finds advancing together, so their
// loads overlap, by path halving: x moves to its grandparent, which also
// becomes its parent. Faster for the waterfall's region unions, whose paths
// are longer; slower for the watershed's short crossing paths.
__device__ __forceinline__ void gunion_halve(int32_t *par, int32_t a, int32_t b) {
    for (;;) {
        for (;;) {
            const int32_t pa = ld_par(par + a), pb = ld_par(par + b);
            if (pa == a && pb == b) break;
            const int32_t ppa = ld_par(par + pa), ppb = ld_par(par + pb);
            if (pa != a) {
                if (ppa != pa) __hip_atomic_store(par + a, ppa, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
                a = ppa;
            }
            if (pb != b) {
                if (ppb != pb) __hip_atomic_store(par + b, ppb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
                b = ppb;
            }
        }
        if (a == b) return;
        if (a < b) {
            const int32_t t = a;
            a = b;
            b = t;
        }
        const int32_t old = atomicCAS(par + a, a, b);
        if (old == a) return;
        a = old;  // a was hooked meanwhile: continue from its new parent
    }
}

// Same union-find on a tile-local parent array in LDS.
__device__ __forceinline__ int lfind(int *par, int x) {
    for (;;) {
        int px = par[x];
        if (px == x) return x;
        int ppx = par[px];
        if (ppx != px) par[x] = ppx;
        x = px;
    }
}

__device__ __forceinline__ void lunion(int *par, int a, int b) {
    a = lfind(par, a);
    b = lfind(par, b);
    while (a != b) {
        if (a < b) { int t = a; a = b; b = t; }
        int old = atomicCAS(par + a, a, b);
        if (old == a) return;
        a = lfind(par, old);
        b = lfind(par, b);
    }
}

// Appends `value` to list[] for every lane with pred set; one atomic per wave.
__device__ __forceinline__ void wave_append(bool pred, int32_t value, int32_t *list, int32_t *counter) {
    uint64_t m = __ballot(pred);
    if (m == 0) return;
    int lane = __lane_id();
    int leader = __ffsll((unsigned long long)m) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(counter, __popcll(m));
    base = __shfl(base, leader);
    if (pred) list[base + __popcll(m & ((1ull << lane) - 1ull))] = value;
}

}  // namespace wsk
