// ws_tiles.h -- gfx950 tile kernels of the watershed transform (Alg. 1),
// templated on the tile shape (shape ids of TileShape in ws_device.h); every
// shape is instantiated in a translation unit of its own (ws_shape.hip).
//
// Data on the device (int32 unless noted, per image):
//   I  grey values (uint8/uint16), read only
//   D  Step II distance field (arena-wide scratch): 0 for pixels with a lower
//      neighbour (state 0) and for strict local minima (state 1); d >= 1 for a
//      non-minimal plateau pixel at geodesic distance d from its plateau's
//      lower border; INF for pixels of minimal plateaux (states 2/3 that Step
//      II never resolves).
//   L  labels / union-find parents (parent <= pixel, roots are self loops).
//
// Step II is computed as the unique fixpoint of
//   D(p) = 1 + min{ D(q) : q in N(p), I(q) = I(p) }      (plateau pixels)
// which both the synchronous sweeps of Section 3.3 and the balanced
// block-asynchronous sweeps of Section 3.4 (Alg. 3) converge to. Tiles relax
// to a local fixpoint in LDS with frozen halos; a tile re-runs only when a
// neighbouring tile changed border distances next to it (tile "stamps" with
// the faces that changed).
//
// Arrows (Eq. (1) for pixels with a lower neighbour; the equal neighbour at
// distance d-1 with the smallest index for resolved plateau pixels) are then
// contracted inside each tile by path-halving Finds (Step III), minimal plateaux
// are joined by union-find (Step IV), and every tile-local component is named
// by its smallest pixel. Crossings between tiles go through a global
// union-find that always hooks the larger root below the smaller, so every
// basin ends with its smallest pixel index as root: the canonical label.
//
// Every tile kernel handles one tile per workgroup, of one image or of a batch
// of images (through a tile -> image table); the same code serves both.
#pragma once

#include <type_traits>

#include "ws_device.h"
#include "ws_kernels.h"

namespace wsk {

// LDS cells of grey values: 16-bit for uint8 images (out-of-image sentinel
// 0x100, above every uint8 value), int32 for uint16 images (SENT, above every
// uint16 value). Smaller cells let more 3D tiles share a CU's LDS.
template <typename T> struct GreyCell { using type = int; };
template <> struct GreyCell<uint8_t> { using type = uint16_t; };
template <typename GC> __host__ __device__ constexpr int sent_of() { return sizeof(GC) == 2 ? 0x100 : SENT; }

// Loads grey values of the tile plus a ring of width R into LDS; cells
// outside the image get the sentinel.
template <int SH, int R, typename T, typename GC>
__device__ __forceinline__ void load_grey(const Geom &g, const T *__restrict__ I, GC *sI, int ox, int oy, int oz) {
    using S = Lds<SH, R>;
    load_box<S::SX, S::SY, S::SZ, T, GC>(g, ox - R, oy - R, oz - S::RZ, I, sI, (GC)sent_of<GC>());
}

// Loads D of the tile plus a ring of width 1; cells outside the image get INF.
template <int SH>
__device__ __forceinline__ void load_dist(const Geom &g, const int32_t *__restrict__ D, int *sD, int ox, int oy, int oz) {
    using S = Lds<SH, 1>;
    load_box<S::SX, S::SY, S::SZ, int32_t, int>(g, ox - 1, oy - 1, oz - S::RZ, D, sD, INF);
}

// Grey values and D of the tile plus a ring of width 1 in one batch of loads
// (one wait for both arrays instead of one each); cells outside the image get
// SENT and INF.
template <int SH, typename T, typename GC>
__device__ __forceinline__ void load_grey_dist(const Geom &g, const T *__restrict__ I, const int32_t *__restrict__ D,
                                               GC *sI, int *sD, int ox, int oy, int oz) {
    using S = Lds<SH, 1>;
    constexpr int PER = (S::CELLS + NTHREADS - 1) / NTHREADS;
    T v[PER];
    int32_t d[PER];
    const uint64_t okm = box_cells<S::SX, S::SY, S::SZ, PER>(g, ox - 1, oy - 1, oz - S::RZ, [&](int j, int32_t i) {
        v[j] = I[i];
        d[j] = D[i];
    });
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        int c = threadIdx.x + j * NTHREADS;
        if (c < S::CELLS) {
            bool ok = okm >> j & 1u;
            sI[c] = ok ? (GC)v[j] : (GC)sent_of<GC>();
            sD[c] = ok ? d[j] : INF;
        }
    }
}

// Unresolved distance in an LDS distance cell: INF in int32 cells; 0xffff in
// the 16-bit cells of the initial tile pass, whose finite distances never
// exceed the tile's pixel count (its ring holds 0 or unresolved only).
template <typename DC> __device__ __forceinline__ constexpr int dinf_of() { return sizeof(DC) == 2 ? 0xffff : INF; }

// Smallest of d and 1 + the distance of every equal-grey neighbour of LDS
// cell s, branch-free: in unsigned arithmetic an unresolved neighbour
// (INF + 1 or 0xffff + 1) lands above every finite candidate and above d.
template <int CONN, class S, typename GC, typename DC>
__device__ __forceinline__ int relax_best(const GC *sI, const DC *sD, int s, int v, int d) {
    uint32_t best = (uint32_t)d;
#pragma unroll
    for (int k = 0; k < CONN; ++k) {
        const int o = s + S::template off<CONN>(k);
        const uint32_t c = (uint32_t)sD[o] + 1u;
        best = ((int)sI[o] == v && c < best) ? c : best;
    }
    return (int)best;
}

// Relaxes the plateau distances of the tile's pixels to a local fixpoint
// (ring cells frozen). Returns after an iteration in which no thread changed
// anything. Gauss-Seidel order inside LDS; any order reaches the same fixpoint
// because distances only decrease and every value stays an upper bound.
template <int SH, int CONN, int R, typename GC, typename DC>
__device__ __forceinline__ void relax_tile(const GC *sI, DC *sD) {
    using TS = TileShape<SH>;
    using S = Lds<SH, R>;
    constexpr int PIX = TS::X * TS::Y * TS::Z;
    for (;;) {
        int changed = 0;
        for (int i = threadIdx.x; i < PIX; i += NTHREADS) {
            int x = i % TS::X, y = (i / TS::X) % TS::Y, z = i / (TS::X * TS::Y);
            int s = S::at(x, y, z);
            int d = sD[s];
            if (d == 0) continue;          // fixed (lower neighbour / minimum) or
            int v = sI[s];                 // out of image (d == INF, v == sentinel)
            if (v == sent_of<GC>()) continue;
            const int best = relax_best<CONN, S>(sI, sD, s, v, d);
            if (best < d) { sD[s] = (DC)best; changed = 1; }
        }
        if (!__syncthreads_or(changed)) break;
    }
}

// Faces of the tile a pixel lies on: bit 0 / 1 the low / high x face, 2 / 3
// y, 4 / 5 z.
template <int SH>
__device__ __forceinline__ uint32_t face_bits(int x, int y, int z) {
    using TS = TileShape<SH>;
    uint32_t b = (x == 0 ? 1u : 0u) | (x == TS::X - 1 ? 2u : 0u) | (y == 0 ? 4u : 0u) | (y == TS::Y - 1 ? 8u : 0u);
    if (shape_ndim<SH>() == 3) b |= (z == 0 ? 16u : 0u) | (z == TS::Z - 1 ? 32u : 0u);
    return b;
}

// Faces across which a border pixel's new distance d can shorten a neighbour's:
// for every neighbour q of the pixel (LDS cell sc) outside the tile, with the
// same grey value and a ring distance above d + 1 (the ring holds upper
// bounds: distances only decrease), the faces that step crosses. A tile whose
// neighbours report no such face cannot change in the next sweep.
template <int SH, int CONN, int R, typename GC, typename DC>
__device__ __forceinline__ uint32_t cross_faces(const GC *sI, const DC *sD, int sc, int x, int y, int z, int d) {
    using TS = TileShape<SH>;
    using S = Lds<SH, R>;
    const int v = sI[sc];
    uint32_t b = 0;
#pragma unroll
    for (int k = 0; k < CONN; ++k) {
        const int dx = nb_dx<CONN>(k), dy = nb_dy<CONN>(k), dz = nb_dz<CONN>(k);
        const int xx = x + dx, yy = y + dy, zz = z + dz;
        const bool out = xx < 0 || xx >= TS::X || yy < 0 || yy >= TS::Y || zz < 0 || zz >= TS::Z;
        if (!out) continue;
        const int o = sc + S::template off<CONN>(k);
        // both reads unconditional (no branch per neighbour); d + 1 cannot
        // overflow: d < INF here
        const int wi = sI[o], wd = sD[o];
        const uint32_t f = (xx < 0 ? 1u : 0u) | (xx >= TS::X ? 2u : 0u) | (yy < 0 ? 4u : 0u) | (yy >= TS::Y ? 8u : 0u) |
                           (zz < 0 ? 16u : 0u) | (zz >= TS::Z ? 32u : 0u);
        b |= ((wi == v) & (wd > d + 1)) ? f : 0u;
    }
    return b;
}

template <int SH>
__device__ __forceinline__ void tile_pixel(int i, int &x, int &y, int &z) {
    using TS = TileShape<SH>;
    x = i % TS::X;
    y = (i / TS::X) % TS::Y;
    z = i / (TS::X * TS::Y);
}

template <int SH>
__device__ __forceinline__ void ws_tile(const Geom &g, int lt, int &ox, int &oy, int &oz) {
    using TS = TileShape<SH>;
    tile_xyz<TS::X, TS::Y, TS::Z>(g, lt, ox, oy, oz);
}

// Step II relaxes only the pixels whose distance can still change: the
// unresolved plateau pixels of a tile are compacted once into an LDS list (in
// index order), and every relaxation pass visits the list instead of the whole
// tile. Plateau pixels are a few per cent of a tile on natural gradients; a
// tile with more than lcap<SH>() of them (LPER entries per thread) relaxes the
// whole tile instead.
template <int SH> __host__ __device__ constexpr int lcap() { return TileShape<SH>::LPER * NTHREADS; }

// Tile pixels i in the image and with (sweep ? D != 0 : D == INF) into lst, in
// index order; returns their number (entries beyond lcap are not stored).
template <int SH, int R, typename GC, typename DC>
__device__ __forceinline__ int build_list(const GC *sI, const DC *sD, unsigned short *lst, bool sweep) {
    using TS = TileShape<SH>;
    using S = Lds<SH, R>;
    constexpr int PIX = TS::X * TS::Y * TS::Z;
    constexpr int PER = PIX / NTHREADS;
    static_assert(PIX % NTHREADS == 0 && PER <= 32, "pixels per thread fit one mask");
    uint32_t m = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        int x, y, z;
        tile_pixel<SH>(threadIdx.x + j * NTHREADS, x, y, z);
        int sc = S::at(x, y, z), d = sD[sc];
        bool take = (int)sI[sc] != sent_of<GC>() && (sweep ? d != 0 : d == dinf_of<DC>());
        m |= (take ? 1u : 0u) << j;
    }
    int excl;
    const int total = block_scan_excl(__popc(m), excl);
    if (total <= lcap<SH>()) {
#pragma unroll
        for (int j = 0; j < PER; ++j)
            if (m >> j & 1u) lst[excl++] = (unsigned short)(threadIdx.x + j * NTHREADS);
    }
    __syncthreads();
    return total;
}

// The listed pixels of this thread: entries threadIdx.x + j * NTHREADS,
// j < LPER, with their LDS cell (-1 past the list) and grey value.
template <int SH, int R, typename GC>
struct ListSlots {
    static constexpr int LP = TileShape<SH>::LPER;
    int sc[LP], v[LP], x[LP], y[LP], z[LP];
    __device__ __forceinline__ void load(const GC *sI, const unsigned short *lst, int n) {
        using S = Lds<SH, R>;
#pragma unroll
        for (int j = 0; j < LP; ++j) {
            const int e = threadIdx.x + j * NTHREADS;
            x[j] = y[j] = z[j] = 0;
            sc[j] = -1;
            v[j] = 0;
            if (e < n) {
                tile_pixel<SH>(lst[e], x[j], y[j], z[j]);
                sc[j] = S::at(x[j], y[j], z[j]);
                v[j] = sI[sc[j]];
            }
        }
    }
};

// relax_tile restricted to the n <= lcap listed pixels.
template <int SH, int CONN, int R, typename GC, typename DC>
__device__ __forceinline__ void relax_list(const GC *sI, DC *sD, const ListSlots<SH, R, GC> &ls) {
    using S = Lds<SH, R>;
    for (;;) {
        int changed = 0;
#pragma unroll
        for (int j = 0; j < ListSlots<SH, R, GC>::LP; ++j) {
            if (ls.sc[j] >= 0) {
                const int d = sD[ls.sc[j]], best = relax_best<CONN, S>(sI, sD, ls.sc[j], ls.v[j], d);
                if (best < d) {
                    sD[ls.sc[j]] = (DC)best;
                    changed = 1;
                }
            }
        }
        if (!__syncthreads_or(changed)) break;
    }
}

// Stamps are double-buffered by sweep parity: stamp[(s & 1) * n + t] holds
// the last sweep of parity s & 1 in which tile t changed distances that a
// neighbour can use, stamp[(2 + (s & 1)) * n + t] the faces concerned. Sweep s
// reads only the buffers of sweep s - 1, which no tile writes during sweep s
// (with one buffer, a neighbour that re-stamped earlier in the same sweep hid
// its previous sweep's faces from the tiles next to them).
__device__ __forceinline__ int32_t *stamp_of(int32_t *stamp, int32_t n, int32_t s) { return stamp + (size_t)(s & 1) * n; }
__device__ __forceinline__ int32_t *faces_of(int32_t *stamp, int32_t n, int32_t s) {
    return stamp + (size_t)(2 + (s & 1)) * n;
}

// Tile t changed border distances in sweep s: record s and the faces.
__device__ __forceinline__ void stamp_tile(int *smk, int32_t *stamp, int32_t n, int32_t *changed, int t, int32_t s,
                                           uint32_t faces) {
    if (faces) atomicOr(smk, (int)faces);
    __syncthreads();
    if (threadIdx.x == 0 && *smk) {
        stamp_of(stamp, n, s)[t] = s;
        faces_of(stamp, n, s)[t] = *smk;
        atomicAdd(changed, 1);
    }
}

// ---------------------------------------------------------------------------
// Step I + first Step II pass: initial distances of the tile and its ring
// (0 = has a lower neighbour or no equal one, INF = plateau pixel), then a
// local fixpoint. Stamps the tile with sweep 0, and the faces concerned, when
// a border pixel obtained a finite distance its neighbours could not have
// known.
// ---------------------------------------------------------------------------
template <int SH, int CONN, typename T, class Src>
__global__ __launch_bounds__(NTHREADS) void k_ws_init(Src src, int32_t ntiles, int32_t *__restrict__ Darena,
                                                      int32_t *__restrict__ stamp, int32_t *__restrict__ changed) {
    using TS = TileShape<SH>;
    using S2 = Lds<SH, 2>;
    using S1 = Lds<SH, 1>;
    constexpr int PIX = TS::X * TS::Y * TS::Z;
    using GC = typename GreyCell<T>::type;
    // Volumes keep 16-bit distance cells (the finite distances of the tile
    // pass stay below the tile's pixel count) to fit more workgroups per CU;
    // 2D tiles already fit eight with int32 cells, and their 16-bit LDS
    // accesses measured slower on plateau-heavy tiles.
    using DC = typename std::conditional<shape_ndim<SH>() == 3, uint16_t, int>::type;
    static_assert(PIX < 0xffff, "16-bit distance cells");
    __shared__ GC sI[S2::CELLS];
    __shared__ DC sD[S2::CELLS];
    __shared__ unsigned short lst[lcap<SH>()];
    __shared__ int smk;
    {
        if ((int)blockIdx.x >= ntiles) return;
        const int t = xcd_tile(blockIdx.x, ntiles);
        Img im;
        int lt;
        fetch(src, t, TK_WS, im, lt);
        const Geom &g = im.g;
        int32_t *D = Darena + im.pix0;
        int ox, oy, oz;
        ws_tile<SH>(g, lt, ox, oy, oz);
        if (threadIdx.x == 0) smk = 0;
        load_grey<SH, 2, T>(g, (const T *)im.grey, sI, ox, oy, oz);
        __syncthreads();
        // Initial distances on the tile plus a ring of width 1 (Step I state test).
        // (An unrolled form with stepped coordinates measured slower.)
        for (int c = threadIdx.x; c < S1::CELLS; c += NTHREADS) {
            int cx = c % S1::SX, cy = (c / S1::SX) % S1::SY, cz = c / (S1::SX * S1::SY);
            int s = S2::at(cx - 1, cy - 1, cz - S1::RZ);
            int v = sI[s];
            int d = dinf_of<DC>();
            if (v != sent_of<GC>()) {
                int m = sent_of<GC>();
#pragma unroll
                for (int k = 0; k < CONN; ++k) m = min(m, (int)sI[s + S2::template off<CONN>(k)]);
                d = (m == v) ? dinf_of<DC>() : 0;
            }
            sD[s] = (DC)d;
        }
        __syncthreads();
        const int n = build_list<SH, 2>(sI, sD, lst, false);
        if (n <= lcap<SH>()) {
            ListSlots<SH, 2, GC> ls;
            ls.load(sI, lst, n);
            relax_list<SH, CONN, 2>(sI, sD, ls);
        } else {
            relax_tile<SH, CONN, 2>(sI, sD);
        }
        uint32_t faces = 0;
        for (int i = threadIdx.x; i < PIX; i += NTHREADS) {
            int x, y, z;
            tile_pixel<SH>(i, x, y, z);
            int gx = ox + x, gy = oy + y, gz = oz + z;
            if (!in_image(g, gx, gy, gz)) continue;
            const int sc = S2::at(x, y, z);
            int d = sD[sc];
            const bool fin = d != dinf_of<DC>();
            D[gx + g.nx * (gy + g.ny * gz)] = fin ? d : INF;
            if (d != 0 && fin && face_bits<SH>(x, y, z)) faces |= cross_faces<SH, CONN, 2>(sI, sD, sc, x, y, z, d);
        }
        stamp_tile(&smk, stamp, ntiles, changed, t, 0, faces);
    }
}

// ---------------------------------------------------------------------------
// Step II sweep s >= 1: tiles next to a tile that changed, in sweep s-1, the
// distances on the face (4/6-connectivity) or anywhere on the border (8/26)
// next to them reload their ring from global memory and relax again.
// ---------------------------------------------------------------------------
template <int SH, int CONN, typename T, class Src>
__global__ __launch_bounds__(NTHREADS) void k_ws_sweep(Src src, int32_t ntiles, int32_t *__restrict__ Darena,
                                                       int32_t *__restrict__ stamp, int32_t *__restrict__ changed,
                                                       const int32_t *__restrict__ prev, int32_t s) {
    using TS = TileShape<SH>;
    using S = Lds<SH, 1>;
    constexpr int PIX = TS::X * TS::Y * TS::Z;
    constexpr int PER = (PIX + NTHREADS - 1) / NTHREADS;
    constexpr bool FACES = CONN == 4 || CONN == 6;  // only face neighbours interact
    using GC = typename GreyCell<T>::type;
    __shared__ GC sI[S::CELLS];
    __shared__ int sD[S::CELLS];
    __shared__ unsigned short lst[lcap<SH>()];
    __shared__ int smk;
    {
        // no tile changed in sweep s - 1 (its counter is final: the launches
        // are ordered on the stream): nothing can change now
        if ((int)blockIdx.x >= ntiles || *prev == 0) return;
        const int t = xcd_tile(blockIdx.x, ntiles);
        Img im;
        int lt;
        fetch(src, t, TK_WS, im, lt);
        const Geom &g = im.g;
        int tx = lt % g.ntx, ty = (lt / g.ntx) % g.nty, tz = lt / (g.ntx * g.nty);
        int active = 0;
        {
            int j = threadIdx.x;  // one neighbouring tile per thread
            if (j < 27) {
                int dx = j % 3 - 1, dy = (j / 3) % 3 - 1, dz = j / 9 - 1;
                int ux = tx + dx, uy = ty + dy, uz = tz + dz;
                bool face = (dx != 0) + (dy != 0) + (dz != 0) == 1;
                bool used = (shape_ndim<SH>() == 3 || dz == 0) && (dx != 0 || dy != 0 || dz != 0) && (!FACES || face);
                if (used && ux >= 0 && ux < g.ntx && uy >= 0 && uy < g.nty && uz >= 0 && uz < g.ntz) {
                    int32_t u = im.tile0[TK_WS] + ux + g.ntx * (uy + g.nty * uz);
                    if (stamp_of(stamp, ntiles, s - 1)[u] == s - 1) {
                        // the neighbour's face towards this tile
                        uint32_t need = !FACES ? 63u
                                        : dx > 0 ? 1u : dx < 0 ? 2u : dy > 0 ? 4u : dy < 0 ? 8u : dz > 0 ? 16u : 32u;
                        active = ((uint32_t)faces_of(stamp, ntiles, s - 1)[u] & need) != 0;
                    }
                }
            }
        }
        if (!__syncthreads_or(active)) return;
        if (threadIdx.x == 0) smk = 0;
        int32_t *D = Darena + im.pix0;
        int ox = tx * TS::X, oy = ty * TS::Y, oz = tz * TS::Z;
        load_grey_dist<SH, T>(g, (const T *)im.grey, D, sI, sD, ox, oy, oz);
        __syncthreads();
        const int n = build_list<SH, 1>(sI, sD, lst, true);
        uint32_t faces = 0;
        if (n <= lcap<SH>()) {
            ListSlots<SH, 1, GC> ls;
            ls.load(sI, lst, n);
            constexpr int LP = ListSlots<SH, 1, GC>::LP;
            int before[LP];
#pragma unroll
            for (int j = 0; j < LP; ++j) before[j] = ls.sc[j] >= 0 ? sD[ls.sc[j]] : 0;
            relax_list<SH, CONN, 1>(sI, sD, ls);
#pragma unroll
            for (int j = 0; j < LP; ++j) {
                if (ls.sc[j] < 0) continue;
                const int d = sD[ls.sc[j]];
                if (d != before[j]) {
                    const int x = ls.x[j], y = ls.y[j], z = ls.z[j];
                    D[(ox + x) + g.nx * ((oy + y) + g.ny * (oz + z))] = d;  // listed pixels are in the image
                    if (face_bits<SH>(x, y, z)) faces |= cross_faces<SH, CONN, 1>(sI, sD, ls.sc[j], x, y, z, d);
                }
            }
        } else {
            int before[PER];
#pragma unroll
            for (int j = 0; j < PER; ++j) {
                int i = threadIdx.x + j * NTHREADS;
                before[j] = INF;
                if (i < PIX) {
                    int x, y, z;
                    tile_pixel<SH>(i, x, y, z);
                    before[j] = sD[S::at(x, y, z)];
                }
            }
            relax_tile<SH, CONN, 1>(sI, sD);
#pragma unroll
            for (int j = 0; j < PER; ++j) {
                int i = threadIdx.x + j * NTHREADS;
                if (i >= PIX) continue;
                int x, y, z;
                tile_pixel<SH>(i, x, y, z);
                int gx = ox + x, gy = oy + y, gz = oz + z;
                if (!in_image(g, gx, gy, gz)) continue;
                const int sc = S::at(x, y, z);
                int d = sD[sc];
                if (d != before[j]) {
                    D[gx + g.nx * (gy + g.ny * gz)] = d;
                    if (face_bits<SH>(x, y, z)) faces |= cross_faces<SH, CONN, 1>(sI, sD, sc, x, y, z, d);
                }
            }
        }
        stamp_tile(&smk, stamp, ntiles, changed, t, s, faces);
    }
}

// ---------------------------------------------------------------------------
// Arrow of one pixel from LDS (ring width 1). Returns the neighbour index k
// the pixel points to, -1 for a root (local minimum), -2 for a minimal
// plateau pixel (joined with its equal neighbours instead).
// ---------------------------------------------------------------------------
template <int SH, int CONN, typename GC>
__device__ __forceinline__ int lds_arrow(const GC *sI, const int *sD, int s) {
    using S = Lds<SH, 1>;
    int v = sI[s], d = sD[s];
    if (d == INF) return -2;
    if (d == 0) {
        int m = sent_of<GC>(), kq = -1;
#pragma unroll
        for (int k = 0; k < CONN; ++k) {
            int w = sI[s + S::template off<CONN>(k)];  // promoted to int
            if (w <= m) { m = w; kq = k; }     // Eq. (1): last of the lowest
        }
        return (m < v) ? kq : -1;
    }
    // first (smallest index) equal neighbour one step closer; all neighbours
    // are read, without an early exit (no per-neighbour branch), and the
    // reverse order leaves the smallest match. -1 is unreachable for a
    // converged distance field.
    int ke = -1;
#pragma unroll
    for (int k = CONN - 1; k >= 0; --k) {
        const int o = s + S::template off<CONN>(k);
        const int wi = sI[o], wd = sD[o];
        if ((wi == v) & (wd == d - 1)) ke = k;  // both reads unconditional: no branch per neighbour
    }
    return ke;
}

// ---------------------------------------------------------------------------
// Border cells of a tile: NB(2D) = 2X + 2(Y-2), NB(3D) = 2XY + (Z-2)(2X +
// 2(Y-2)). A tile's crossing records take RS = NB + 1 ints: a count, then at
// most one entry per border cell (only border pixels have a neighbour outside
// the tile).
// ---------------------------------------------------------------------------
template <int SH> struct Border {
    using TS = TileShape<SH>;
    static constexpr int RING = 2 * TS::X + 2 * (TS::Y - 2);
    static constexpr int FACE = TS::X * TS::Y;
    static constexpr int NB = shape_ndim<SH>() == 2 ? RING : 2 * FACE + (TS::Z - 2) * RING;
    static constexpr int RS = NB + 1;
};

// A crossing record: the in-tile index of the smallest pixel of the pixel's
// tile-local component (bits 17..28), the pixel's in-tile index (5..16) and
// the neighbour its arrow leaves the tile through, or REC_PLATEAU for a
// minimal-plateau pixel with an equal neighbour outside the tile (after it in
// the neighbourhood order) (0..4). Tiles hold at most 4096 pixels.
constexpr int REC_PLATEAU = 31;
__host__ __device__ constexpr int32_t rec_entry(int i, int k) { return (int32_t)((i << 5) | k); }
__host__ __device__ constexpr int32_t rec_with_min(int32_t e, int cm) { return (int32_t)(cm << 17) | e; }

// ---------------------------------------------------------------------------
// Tile-local labelling. Every pixel's arrow inside the tile is contracted (a
// Find with path halving, Step III) to its terminal: a local minimum,
// a minimal-plateau pixel, or an exit whose arrow leaves the tile. Minimal-
// plateau pixels are then joined with their equal neighbours by union-find
// (Step IV). Each tile-local component is named by its smallest pixel (LDS
// atomicMin), written into L. The crossings the global merge needs are
// appended to the tile's records (rec_entry): every arrow that leaves the
// tile, and every minimal-plateau pixel with an equal neighbour outside it.
// ---------------------------------------------------------------------------
template <int SH, int CONN, typename T, class Src>
__global__ __launch_bounds__(NTHREADS) void k_ws_label(Src src, int32_t ntiles, const int32_t *__restrict__ Darena,
                                                       int32_t *__restrict__ rec) {
    using TS = TileShape<SH>;
    using S = Lds<SH, 1>;
    constexpr int PIX = TS::X * TS::Y * TS::Z;
    constexpr int PER = PIX / NTHREADS;
    static_assert(PIX % NTHREADS == 0, "tile must be a multiple of the workgroup");
    static_assert(S::CELLS >= PIX, "the parent array fits the distance array");
    using GC = typename GreyCell<T>::type;
    // two LDS arrays: grey values, and distances that become the tile's
    // parent array once every arrow is known
    __shared__ GC sI[S::CELLS];
    __shared__ int sD[S::CELLS];
    __shared__ int nrec;
    int *sP = sD;
    {
        if ((int)blockIdx.x >= ntiles) return;
        if (threadIdx.x == 0) nrec = 0;
        const int t = xcd_tile(blockIdx.x, ntiles);
        Img im;
        int lt;
        fetch(src, t, TK_WS, im, lt);
        const Geom &g = im.g;
        int32_t *L = im.lab;
        int ox, oy, oz;
        ws_tile<SH>(g, lt, ox, oy, oz);
        load_grey_dist<SH, T>(g, (const T *)im.grey, Darena + im.pix0, sI, sD, ox, oy, oz);
        __syncthreads();
        uint32_t minzone = 0, inimg = 0;
        int tos[PER];
        int32_t *trec = rec + (size_t)t * Border<SH>::RS;
        static_assert(PIX <= 4096, "in-tile indices fit the records' 12-bit fields");
        int32_t ents[PER];  // crossing record of each pixel (without its component), -1 if none
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            int i = threadIdx.x + j * NTHREADS;
            int x = i % TS::X, y = (i / TS::X) % TS::Y, z = i / (TS::X * TS::Y);
            int gx = ox + x, gy = oy + y, gz = oz + z;
            int to = i;
            int32_t ent = -1;  // crossing record of this pixel, if any
            if (in_image(g, gx, gy, gz)) {
                inimg |= 1u << j;
                int s = S::at(x, y, z);
                int k = lds_arrow<SH, CONN>(sI, sD, s);
                if (k >= 0) {
                    int xx = x + nb_dx<CONN>(k), yy = y + nb_dy<CONN>(k), zz = z + nb_dz<CONN>(k);
                    if (xx >= 0 && xx < TS::X && yy >= 0 && yy < TS::Y && zz >= 0 && zz < TS::Z)
                        to = xx + TS::X * (yy + TS::Y * zz);
                    else
                        ent = rec_entry(i, k);
                } else if (k == -2) {
                    minzone |= 1u << j;
                    int v = sI[s];
#pragma unroll
                    for (int k2 = CONN / 2; k2 < CONN; ++k2) {  // neighbours after p
                        int xx = x + nb_dx<CONN>(k2), yy = y + nb_dy<CONN>(k2), zz = z + nb_dz<CONN>(k2);
                        bool inside = xx >= 0 && xx < TS::X && yy >= 0 && yy < TS::Y && zz >= 0 && zz < TS::Z;
                        if (!inside && sI[s + S::template off<CONN>(k2)] == v) ent = rec_entry(i, REC_PLATEAU);
                    }
                }
            }
            ents[j] = ent;
            tos[j] = to;
        }
        __syncthreads();  // every distance read: the array becomes the parents
#pragma unroll
        for (int j = 0; j < PER; ++j) sP[threadIdx.x + j * NTHREADS] = tos[j];
        __syncthreads();
        // The arrows form an in-tile forest whose roots are the terminals (a
        // local minimum, a minimal-plateau pixel, or an exit); the Finds below
        // reach them, halving the paths they walk (Step III inside the tile).
        // Minimal plateaux: join equal neighbours after p inside the tile.
        // Minimal-plateau pixels are few (about 1.6 % on the volume recipe) and
        // scattered over the thread's PER pixels: each thread walks only its
        // own, so the wave runs as many rounds as its busiest lane has pixels
        // (mostly one or two) instead of one round per j.
        {
            uint32_t mz = minzone;
            while (mz) {
                const int j = __ffs(mz) - 1;
                mz &= mz - 1;
                int i = threadIdx.x + j * NTHREADS;
                int x = i % TS::X, y = (i / TS::X) % TS::Y, z = i / (TS::X * TS::Y);
                int s = S::at(x, y, z);
                int v = sI[s];
#pragma unroll
                for (int k2 = CONN / 2; k2 < CONN; ++k2) {
                    int xx = x + nb_dx<CONN>(k2), yy = y + nb_dy<CONN>(k2), zz = z + nb_dz<CONN>(k2);
                    if (xx < 0 || xx >= TS::X || yy < 0 || yy >= TS::Y || zz < 0 || zz >= TS::Z) continue;
                    if (sI[s + S::template off<CONN>(k2)] == v) lunion(sP, i, xx + TS::X * (yy + TS::Y * zz));
                }
            }
        }
        __syncthreads();
        // smallest pixel of every tile-local component, in the root's own
        // parent entry once every root is known: a root holds its own index,
        // and the root of an in-image pixel is itself in the image (arrows and
        // plateau unions never reach a cell outside), so it is a candidate
        // All PER paths of the thread advance together (their LDS reads
        // overlap), each by path halving: x moves to its grandparent, which
        // also becomes its parent.
        int root[PER];
        uint32_t live = 0;
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            root[j] = threadIdx.x + j * NTHREADS;
            live |= 1u << j;
        }
        while (live) {
            int px[PER], ppx[PER];
#pragma unroll
            for (int j = 0; j < PER; ++j) px[j] = sP[root[j]];
#pragma unroll
            for (int j = 0; j < PER; ++j) ppx[j] = sP[px[j]];
            // Branch-free (per-path branches cost scalar exec-mask work): a
            // finished path has px == root and ppx == px (a root's entry
            // never changes here, every union is done), so every path moves
            // to ppx, and the halving store may be unconditional: where
            // ppx == px it writes back the parent read (or, if another lane
            // halved that entry meanwhile, an ancestor of it: still valid).
            uint32_t nl = 0;
#pragma unroll
            for (int j = 0; j < PER; ++j) {
                nl |= (px[j] != root[j] ? 1u : 0u) << j;
                sP[root[j]] = ppx[j];
                root[j] = ppx[j];
            }
            live = nl;
        }
        __syncthreads();
        int *cm = sP;
#pragma unroll
        for (int j = 0; j < PER; ++j)
            if (inimg >> j & 1u) atomicMin(&cm[root[j]], (int)(threadIdx.x + j * NTHREADS));
        __syncthreads();
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int i = threadIdx.x + j * NTHREADS;
            const int r = cm[root[j]];
            if (inimg >> j & 1u) {
                int x = i % TS::X, y = (i / TS::X) % TS::Y, z = i / (TS::X * TS::Y);
                int rx = r % TS::X, ry = (r / TS::X) % TS::Y, rz = r / (TS::X * TS::Y);
                L[(ox + x) + g.nx * ((oy + y) + g.ny * (oz + z))] = (ox + rx) + g.nx * ((oy + ry) + g.ny * (oz + rz));
            }
            // append the wave's records, each with its component's smallest
            // pixel, with one LDS reservation
            const uint64_t m = __ballot(ents[j] >= 0);
            if (m) {  // wave-uniform
                int wbase = 0;
                if (__lane_id() == 0) wbase = atomicAdd(&nrec, __popcll(m));
                wbase = __shfl(wbase, 0);
                if (ents[j] >= 0) trec[1 + wbase + __popcll(m & lanes_below())] = rec_with_min(ents[j], r);
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) trec[0] = nrec;
    }
}

// Union of lp (the tile-pass root of a pixel, from its record) and the root
// L[r] of its neighbour r for the lanes with `want`, once per distinct pair:
// border cells next to each other mostly join the same two tile-local
// components, so a wave first elects one lane per distinct (lp, L[r]) pair
// (ballots, no memory traffic) and only those lanes run the global union, all
// at once.
__device__ __forceinline__ void wave_unique_union(int32_t *L, bool want, int32_t lp, int32_t r) {
    uint64_t pending = __ballot(want);
    if (pending == 0) return;  // wave-uniform
    int32_t a = -1, b = -1;
    if (want) {
        const int32_t lr = ld_par(L + r);
        a = lp < lr ? lp : lr;
        b = lp < lr ? lr : lp;
    }
    bool lead = false;
    while (pending) {
        const int leader = __ffsll((unsigned long long)pending) - 1;
        const int32_t la = __shfl(a, leader), lb = __shfl(b, leader);
        const uint64_t same = __ballot(want && a == la && b == lb);
        if ((int)__lane_id() == leader) lead = true;
        pending &= ~same;
    }
    if (lead && a != b) gunion(L, a, b);
}

// ---------------------------------------------------------------------------
// Unions for every arrow / minimal-plateau adjacency that crosses a tile
// border, driven by the tile's records from k_ws_label: one thread per record.
// Each exit record starts its own tile-local component (an exit is the
// terminal of its in-tile path), so its pair of roots is distinct and it
// unites directly; plateau records of volumes first elect one lane per pair.
// ---------------------------------------------------------------------------
template <int SH, int CONN, typename T, class Src>
__global__ __launch_bounds__(NTHREADS) void k_ws_merge(Src src, int32_t ntiles, const int32_t *__restrict__ rec) {
    using TS = TileShape<SH>;
    constexpr int RS = Border<SH>::RS;
    {
        if ((int)blockIdx.x >= ntiles) return;
        const int t = xcd_tile(blockIdx.x, ntiles);
        Img im;
        int lt;
        fetch(src, t, TK_WS, im, lt);
        const Geom &g = im.g;
        const T *I = (const T *)im.grey;
        int32_t *L = im.lab;
        int ox, oy, oz;
        ws_tile<SH>(g, lt, ox, oy, oz);
        const int32_t *trec = rec + (size_t)t * RS;
        const int n = trec[0];
        for (int e0 = 0; e0 < n; e0 += NTHREADS) {  // uniform trip count
            const int e = e0 + (int)threadIdx.x;
            const int32_t ent = e < n ? trec[1 + e] : -1;
            int gx = 0, gy = 0, gz = 0, k = -1;
            int32_t pm = 0;  // smallest pixel of p's tile-local component (its tile-pass root)
            if (ent >= 0) {
                const int i = (ent >> 5) & 0xfff, c = ent >> 17;
                k = ent & 31;
                gx = ox + i % TS::X;
                gy = oy + (i / TS::X) % TS::Y;
                gz = oz + i / (TS::X * TS::Y);
                pm = (ox + c % TS::X) + g.nx * ((oy + (c / TS::X) % TS::Y) + g.ny * (oz + c / (TS::X * TS::Y)));
            }
            const int32_t p = gx + g.nx * (gy + g.ny * gz);
            if (k >= 0 && k != REC_PLATEAU)
                gunion(L, pm, (gx + nb_dx<CONN>(k)) + g.nx * ((gy + nb_dy<CONN>(k)) + g.ny * (gz + nb_dz<CONN>(k))));
            const bool plat = k == REC_PLATEAU;
            const int v = plat ? (int)I[p] : 0;
#pragma unroll
            for (int k2 = CONN / 2; k2 < CONN; ++k2) {  // equal neighbours after p outside the tile
                int32_t r = -1;
                if (plat) {
                    int xx = gx + nb_dx<CONN>(k2), yy = gy + nb_dy<CONN>(k2), zz = gz + nb_dz<CONN>(k2);
                    bool outside = !(xx >= ox && xx < ox + TS::X && yy >= oy && yy < oy + TS::Y && zz >= oz &&
                                     zz < oz + TS::Z);
                    if (outside && in_image(g, xx, yy, zz)) {
                        int32_t q = xx + g.nx * (yy + g.ny * zz);
                        if ((int)I[q] == v) r = q;
                    }
                }
                // volumes (many plateau records per component pair) elect one
                // lane per pair; 2D tiles measured faster without
                if constexpr (shape_ndim<SH>() == 3) wave_unique_union(L, r >= 0, pm, r);
                else if (r >= 0) gunion(L, pm, r);
            }
        }
    }
}

// Walks r[j] to its root for every j with bit j of `live`, all paths of the
// thread together so that their loads overlap.
template <int PER>
__device__ __forceinline__ void find_walk(const int32_t *L, int32_t (&r)[PER], uint32_t live) {
    while (live) {
        int32_t nxt[PER];
#pragma unroll
        for (int j = 0; j < PER; ++j) nxt[j] = (live >> j & 1u) ? L[r[j]] : r[j];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            if (!(live >> j & 1u)) continue;
            if (nxt[j] == r[j]) live &= ~(1u << j);
            else r[j] = nxt[j];
        }
    }
}

// ---------------------------------------------------------------------------
// Final Find of every pixel (APRUF form: every pixel, or in volumes one pixel
// per tile-local component name, follows its path to the root), per
// watershed tile.
// ---------------------------------------------------------------------------
template <int SH, class Src>
__global__ __launch_bounds__(NTHREADS) void k_ws_find(Src src, int32_t ntiles) {
    using TS = TileShape<SH>;
    constexpr int PIX = TS::X * TS::Y * TS::Z;
    constexpr int PER = PIX / NTHREADS;
    {
        if ((int)blockIdx.x >= ntiles) return;
        const int t = xcd_tile(blockIdx.x, ntiles);
        Img im;
        int lt;
        fetch(src, t, TK_WS, im, lt);
        const Geom &g = im.g;
        int32_t *L = im.lab;
        int ox, oy, oz;
        ws_tile<SH>(g, lt, ox, oy, oz);
        int32_t p[PER], r[PER];
        bool ok[PER];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            int i = threadIdx.x + j * NTHREADS;
            int x = ox + i % TS::X, y = oy + (i / TS::X) % TS::Y, z = oz + i / (TS::X * TS::Y);
            ok[j] = in_image(g, x, y, z);
            p[j] = ok[j] ? x + g.nx * (y + g.ny * z) : 0;
        }
        int32_t l0[PER];
#pragma unroll
        for (int j = 0; j < PER; ++j) r[j] = l0[j] = L[p[j]];
        uint32_t live = 0;
        if constexpr (shape_ndim<SH>() == 3) {
            // Volumes: most pixels still name their tile-local component by
            // its smallest pixel, a pixel of this tile, and paths across tiles
            // are long. One pixel per such name walks to the root (claimed in
            // LDS by the name's in-tile index) and the others read the
            // result; a pixel whose name lies outside the tile walks on its
            // own. (2D tiles measured faster walking every pixel.)
            __shared__ int owner[PIX];
            __shared__ int32_t root_of[PIX];
#pragma unroll
            for (int j = 0; j < PER; ++j) owner[threadIdx.x + j * NTHREADS] = -1;
            __syncthreads();
            int ci[PER];  // in-tile index of the name, -1 outside the tile
#pragma unroll
            for (int j = 0; j < PER; ++j) {
                ci[j] = -1;
                if (!ok[j]) continue;
                int x, y, z;
                pixel_coords(g, l0[j], x, y, z);
                x -= ox;
                y -= oy;
                z -= oz;
                if (x >= 0 && x < TS::X && y >= 0 && y < TS::Y && z >= 0 && z < TS::Z)
                    ci[j] = x + TS::X * (y + TS::Y * z);
                if (ci[j] < 0 || atomicCAS(&owner[ci[j]], -1, (int)threadIdx.x + j * NTHREADS) == -1)
                    live |= 1u << j;
            }
            find_walk<PER>(L, r, live);
#pragma unroll
            for (int j = 0; j < PER; ++j)
                if (ok[j] && ci[j] >= 0 && owner[ci[j]] == (int)threadIdx.x + j * NTHREADS) root_of[ci[j]] = r[j];
            __syncthreads();
#pragma unroll
            for (int j = 0; j < PER; ++j)
                if (ok[j] && ci[j] >= 0) r[j] = root_of[ci[j]];
        } else {
#pragma unroll
            for (int j = 0; j < PER; ++j)
                if (ok[j]) live |= 1u << j;
            find_walk<PER>(L, r, live);
        }
        // a pixel whose label already is its root keeps it (no store)
#pragma unroll
        for (int j = 0; j < PER; ++j)
            if (ok[j] && r[j] != l0[j]) L[p[j]] = r[j];
    }
}

// RR pointer jumps per synchronisation (PRUF form of Step III), per tile.
template <int SH, class Src>
__global__ __launch_bounds__(NTHREADS) void k_ws_jump(Src src, int32_t ntiles, int32_t rr,
                                                      int32_t *__restrict__ changed) {
    using TS = TileShape<SH>;
    constexpr int PIX = TS::X * TS::Y * TS::Z;
    {
        if ((int)blockIdx.x >= ntiles) return;
        const int t = xcd_tile(blockIdx.x, ntiles);
        Img im;
        int lt;
        fetch(src, t, TK_WS, im, lt);
        const Geom &g = im.g;
        int32_t *L = im.lab;
        int ox, oy, oz;
        ws_tile<SH>(g, lt, ox, oy, oz);
        int ch = 0;
        for (int i = threadIdx.x; i < PIX; i += NTHREADS) {
            int x = ox + i % TS::X, y = oy + (i / TS::X) % TS::Y, z = oz + i / (TS::X * TS::Y);
            if (!in_image(g, x, y, z)) continue;
            int32_t p = x + g.nx * (y + g.ny * z);
            int32_t l = L[p];
            bool moved = false;
            for (int k = 0; k < rr; ++k) {
                int32_t ll = ld_par(L + l);
                if (ll == l) break;
                l = ll;
                moved = true;
            }
            if (moved) {
                L[p] = l;
                ch = 1;
            }
        }
        if (__syncthreads_or(ch) && threadIdx.x == 0) atomicAdd(changed, 1);
    }
}

// ---------------------------------------------------------------------------
// Host-side launchers of one shape's tile kernels (instantiated per
// connectivity of the shape's dimensionality, grey type and source).
// ---------------------------------------------------------------------------
template <int SH, int CONN, typename T, class Src>
static int ws_init_t(Launch &lc, const Src &src, const TileGrid &tg, int32_t *D, int32_t *stamp, int32_t *changed) {
    return lc.run("ws_init", k_ws_init<SH, CONN, T, Src>, dim3(tg.grid), dim3(NTHREADS), src, tg.ntiles, D, stamp,
                  changed);
}
template <int SH, int CONN, typename T, class Src>
static int ws_sweep_t(Launch &lc, const Src &src, const TileGrid &tg, int32_t *D, int32_t *stamp, int32_t *changed,
                      const int32_t *prev, int32_t s) {
    return lc.run("ws_sweep", k_ws_sweep<SH, CONN, T, Src>, dim3(tg.grid), dim3(NTHREADS), src, tg.ntiles, D, stamp,
                  changed, prev, s);
}
template <int SH, int CONN, typename T, class Src>
static int ws_label_t(Launch &lc, const Src &src, const TileGrid &tg, const int32_t *D, int32_t *rec) {
    return lc.run("ws_label", k_ws_label<SH, CONN, T, Src>, dim3(tg.grid), dim3(NTHREADS), src, tg.ntiles, D, rec);
}
template <int SH, int CONN, typename T, class Src>
static int ws_merge_t(Launch &lc, const Src &src, const TileGrid &tg, const int32_t *rec) {
    return lc.run("ws_merge", k_ws_merge<SH, CONN, T, Src>, dim3(tg.grid), dim3(NTHREADS), src, tg.ntiles, rec);
}
template <int SH, int CONN, typename T, class Src>
static int ws_find_t(Launch &lc, const Src &src, const TileGrid &tg) {
    return lc.run("ws_find", k_ws_find<SH, Src>, dim3(tg.grid), dim3(NTHREADS), src, tg.ntiles);
}
template <int SH, int CONN, typename T, class Src>
static int ws_jump_t(Launch &lc, const Src &src, const TileGrid &tg, int32_t rr, int32_t *changed) {
    return lc.run("ws_jump", k_ws_jump<SH, Src>, dim3(tg.grid), dim3(NTHREADS), src, tg.ntiles, rr, changed);
}

// Connectivities of the shape's dimensionality; -1 for any other.
#define WS_SHAPE_DISPATCH(FN, conn, u16, ...)                                                                   \
    if constexpr (shape_ndim<SH>() == 2) {                                                                      \
        switch (conn) {                                                                                         \
        case 4: return u16 ? FN<SH, 4, uint16_t>(__VA_ARGS__) : FN<SH, 4, uint8_t>(__VA_ARGS__);               \
        case 8: return u16 ? FN<SH, 8, uint16_t>(__VA_ARGS__) : FN<SH, 8, uint8_t>(__VA_ARGS__);               \
        default: return -1;                                                                                     \
        }                                                                                                       \
    } else {                                                                                                    \
        switch (conn) {                                                                                         \
        case 6: return u16 ? FN<SH, 6, uint16_t>(__VA_ARGS__) : FN<SH, 6, uint8_t>(__VA_ARGS__);               \
        case 26: return u16 ? FN<SH, 26, uint16_t>(__VA_ARGS__) : FN<SH, 26, uint8_t>(__VA_ARGS__);            \
        default: return -1;                                                                                     \
        }                                                                                                       \
    }

#define WS_SHAPE_DEFS(Src)                                                                                          \
    template <int SH>                                                                                               \
    int WsShape<SH>::init(Launch &lc, const Src &src, const TileGrid &tg, int conn, bool u16, int32_t *D,          \
                          int32_t *stamp, int32_t *changed) {                                                       \
        WS_SHAPE_DISPATCH(ws_init_t, conn, u16, lc, src, tg, D, stamp, changed)                                     \
    }                                                                                                               \
    template <int SH>                                                                                               \
    int WsShape<SH>::sweep(Launch &lc, const Src &src, const TileGrid &tg, int conn, bool u16, int32_t *D,         \
                           int32_t *stamp, int32_t *changed, const int32_t *prev, int32_t s) {                      \
        WS_SHAPE_DISPATCH(ws_sweep_t, conn, u16, lc, src, tg, D, stamp, changed, prev, s)                           \
    }                                                                                                               \
    template <int SH>                                                                                               \
    int WsShape<SH>::label(Launch &lc, const Src &src, const TileGrid &tg, int conn, bool u16, const int32_t *D,   \
                           int32_t *rec) {                                                                          \
        WS_SHAPE_DISPATCH(ws_label_t, conn, u16, lc, src, tg, D, rec)                                               \
    }                                                                                                               \
    template <int SH>                                                                                               \
    int WsShape<SH>::merge(Launch &lc, const Src &src, const TileGrid &tg, int conn, bool u16, const int32_t *rec) { \
        WS_SHAPE_DISPATCH(ws_merge_t, conn, u16, lc, src, tg, rec)                                                  \
    }                                                                                                               \
    template <int SH>                                                                                               \
    int WsShape<SH>::find(Launch &lc, const Src &src, const TileGrid &tg, int conn) {                               \
        WS_SHAPE_DISPATCH(ws_find_t, conn, false, lc, src, tg)                                                      \
    }                                                                                                               \
    template <int SH>                                                                                               \
    int WsShape<SH>::jump(Launch &lc, const Src &src, const TileGrid &tg, int conn, int32_t rr, int32_t *changed) { \
        WS_SHAPE_DISPATCH(ws_jump_t, conn, false, lc, src, tg, rr, changed)                                         \
    }

WS_SHAPE_DEFS(OneImg)
WS_SHAPE_DEFS(ImgTable)
#undef WS_SHAPE_DEFS
#undef WS_SHAPE_DISPATCH

template <int SH>
int WsShape<SH>::record_ints() {
    return Border<SH>::RS;
}

}  // namespace wsk
