// ws_kernels.h -- host-side launchers of the libws kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "ws_device.h"

namespace wsk {

// Collects (name, start event, stop event) triples when kernel timing is on.
struct TimingSink {
    struct Rec { std::string name; hipEvent_t a, b; };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    hipEvent_t get() {
        if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
};

// A kernel launch on one stream; records a HIP event pair around it when a
// timing sink is attached. Returns 0 or WS_EDEVICE (-3).
struct Launch {
    hipStream_t stream = nullptr;
    TimingSink *timing = nullptr;
    hipError_t last = hipSuccess;

    template <typename K, typename... A>
    int run(const char *name, K kernel, dim3 grid, dim3 block, A... args) {
        return run_shm(name, kernel, grid, block, 0, args...);
    }

    template <typename K, typename... A>
    int run_shm(const char *name, K kernel, dim3 grid, dim3 block, size_t shm, A... args) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (timing) {
            e0 = timing->get();
            e1 = timing->get();
            if (e0) (void)hipEventRecord(e0, stream);
        }
        hipLaunchKernelGGL(kernel, grid, block, shm, stream, args...);
        hipError_t err = hipGetLastError();
        if (timing && e0 && e1) {
            (void)hipEventRecord(e1, stream);
            timing->recs.push_back({name, e0, e1});
        }
        if (err != hipSuccess) {
            last = err;
            return -3;
        }
        return 0;
    }
};

struct BlurTaps {
    int r;
    float w[129];
};

// Region-id rank tables of the waterfall: per 64 pixels of a chunk, the root
// bitmap word and the id of the first root at or after it; per chunk, its
// first id (the scanned root counts).
struct alignas(16) RankWord {
    unsigned long long bits;
    int32_t base;
    int32_t pad;
};
struct WfIds {
    RankWord *words;
    int32_t *coff;
};

// Tiles of one tiling and the launch grid that covers them (one workgroup per
// tile).
struct TileGrid {
    int32_t ntiles = 0;
    int32_t grid = 0;
};

// The waterfall's per-tile edge slabs: entry j of tile t's slab is the
// region pair p[t * cap + j] (smaller id in the high word) and its pass
// height w[t * cap + j] (grey values are at most 16 bits); cnt[t] holds the
// tile's edge count. 10 bytes per entry. A launch over a sub-range of the
// tiles gets pointers advanced to its first tile (same cap).
struct EdgeSlabs {
    uint64_t *p = nullptr;
    uint16_t *w = nullptr;
    int32_t *cnt = nullptr;
    int32_t cap = 0;
    static constexpr size_t kEntryBytes = 10;
    EdgeSlabs at(int32_t t0) const {
        EdgeSlabs e = *this;
        const size_t o = (size_t)t0 * (size_t)cap;
        e.p += o;
        e.w += o;
        e.cnt += t0;
        return e;
    }
};

// Launchers of the watershed tile kernels of one tile shape (ws_tiles.h),
// instantiated per shape id in ws_shape.hip; conn must have the shape's
// dimensionality (-1 otherwise).
template <int SH>
struct WsShape {
#define WS_SHAPE_SRC(Src)                                                                                        \
    static int init(Launch &lc, const Src &src, const TileGrid &tg, int conn, bool u16, int32_t *D,             \
                    int32_t *stamp, int32_t *changed);                                                           \
    static int sweep(Launch &lc, const Src &src, const TileGrid &tg, int conn, bool u16, int32_t *D,            \
                     int32_t *stamp, int32_t *changed, const int32_t *prev, int32_t s);                          \
    static int label(Launch &lc, const Src &src, const TileGrid &tg, int conn, bool u16, const int32_t *D,      \
                     int32_t *rec);                                                                              \
    static int merge(Launch &lc, const Src &src, const TileGrid &tg, int conn, bool u16, const int32_t *rec);   \
    static int find(Launch &lc, const Src &src, const TileGrid &tg, int conn);                                  \
    static int jump(Launch &lc, const Src &src, const TileGrid &tg, int conn, int32_t rr, int32_t *changed);
    WS_SHAPE_SRC(OneImg)
    WS_SHAPE_SRC(ImgTable)
#undef WS_SHAPE_SRC
    static int record_ints();
};
extern template struct WsShape<2>;
extern template struct WsShape<12>;
extern template struct WsShape<22>;
extern template struct WsShape<32>;
extern template struct WsShape<3>;
extern template struct WsShape<13>;
extern template struct WsShape<23>;
extern template struct WsShape<33>;

// watershed.hip: the tile kernels of any shape id (-1 for an unknown shape or
// a connectivity of the other dimensionality)
#define WS_DECL_SRC(Src)                                                                                          \
    int launch_ws_init(Launch &lc, const Src &src, const TileGrid &tg, int conn, int shape, bool u16, int32_t *D, \
                       int32_t *stamp, int32_t *changed);                                                         \
    int launch_ws_sweep(Launch &lc, const Src &src, const TileGrid &tg, int conn, int shape, bool u16,           \
                        int32_t *D, int32_t *stamp, int32_t *changed, const int32_t *prev, int32_t s);           \
    int launch_ws_label(Launch &lc, const Src &src, const TileGrid &tg, int conn, int shape, bool u16,           \
                        const int32_t *D, int32_t *rec);                                                          \
    int launch_ws_merge(Launch &lc, const Src &src, const TileGrid &tg, int conn, int shape, bool u16,           \
                        const int32_t *rec);                                                                      \
    int launch_ws_find(Launch &lc, const Src &src, const TileGrid &tg, int conn, int shape);                     \
    int launch_ws_jump(Launch &lc, const Src &src, const TileGrid &tg, int conn, int shape, int32_t rr,          \
                       int32_t *changed);                                                                         \
    int launch_wf_ids(Launch &lc, const Src &src_ch, int32_t nchunks, int32_t bound, const WfIds &ids,           \
                      int32_t *scan_tmp, int32_t *nreg0, uint64_t *key, int32_t *par);                            \
    int launch_wf_pix(Launch &lc, const Src &src, const TileGrid &tg, int conn, bool u16, const WfIds &ids,      \
                      const int32_t *nreg0, int32_t *cimg, int32_t *rlist, uint64_t *key, const EdgeSlabs &es);  \
    int launch_wf_out(Launch &lc, const Src &src_ch, int32_t nchunks, int32_t nl, const int32_t *cimg,           \
                      const int32_t *nreg0, const int32_t *coff, const int32_t *mlab, int64_t mstride,          \
                      int64_t hstride, int32_t *cnt);
WS_DECL_SRC(OneImg)
WS_DECL_SRC(ImgTable)
#undef WS_DECL_SRC

int record_ints(int shape);   // record ints per tile of a shape: a count and at most one entry per border cell (0 for an unknown shape)
int launch_ws_stages(Launch &lc, const Geom &g, int conn, bool u16, const void *I, const int32_t *D, int32_t *bal,
                     int32_t *arrow);
int launch_fill_i32(Launch &lc, int32_t *a, int32_t n, int32_t v);
int launch_fill2_i32(Launch &lc, int32_t *a, int32_t na, int32_t va, int32_t *b, int32_t nb, int32_t vb);

// Per-pixel synchronous schedule (one thread per pixel, one launch per step).
int launch_px_step1(Launch &lc, const Geom &g, int conn, bool u16, const void *I, int32_t *L, int32_t *S);
int launch_px_sweep(Launch &lc, const Geom &g, int conn, bool u16, const void *I, int32_t *L, int32_t *S, int32_t s,
                    int32_t *changed);
int launch_px_jump(Launch &lc, const Geom &g, int32_t *L, int32_t rr, int32_t *changed);
int launch_px_find(Launch &lc, const Geom &g, int32_t *L);
int launch_px_union(Launch &lc, const Geom &g, int conn, const int32_t *S, int32_t *L);
int launch_px_prw(Launch &lc, const Geom &g, int conn, const int32_t *S, int32_t *L, int32_t *changed);
int launch_px_canon(Launch &lc, const Geom &g, int32_t *L, int32_t *M);
int launch_px_stages(Launch &lc, const Geom &g, const int32_t *S, int32_t *bal);

// waterfall.hip
int wf_tiles(const Geom &g, int ndim);
int wf_chunks(int32_t n);               // region-id chunks of an image of n pixels
int wf_slab_cap(int conn);              // edge slab entries per tile
int wf_max_merge();                     // largest group merge factor of launch_wf_level
int scan_tmp_len(int32_t n);            // ints of scratch launch_scan needs for n
int launch_scan(Launch &lc, int32_t n, int32_t *data, int32_t *tmp, int32_t *total_out);
int launch_wf_level(Launch &lc, int32_t ntiles, int32_t gin, int32_t f, const int32_t *par, uint64_t *key,
                    const EdgeSlabs &es);
// Layers >= 2 over the layer-1 roots (see waterfall.hip, 2b): the sorted root
// list R1 with ranks in id1 and its length in *n1 (scratch: root_list_tmp_len
// ints); layer 1's compression with ranks; union and compression over R1.
int launch_root_list(Launch &lc, int32_t bound, const int32_t *nreg0, const int32_t *par, int32_t *R1, int32_t *id1,
                     int32_t ids, int32_t cap, int32_t *scratch, int32_t *n1);
int root_list_tmp_len(int32_t bound);
int launch_wf_compress1(Launch &lc, int32_t bound, const int32_t *nreg0, int32_t *par, const int32_t *rlist,
                        int32_t *mlab1, int32_t *id1, int32_t ms);
int launch_wf_union_l(Launch &lc, int32_t bound, const int32_t *n1, int32_t cap, const int32_t *R1, uint64_t *key,
                      int32_t *par);
int launch_wf_compress_l(Launch &lc, int32_t bound, const int32_t *n1, int32_t cap, const int32_t *R1, int32_t *par,
                         const int32_t *rlist, int32_t *Mk, int32_t ls);
int launch_wf_union(Launch &lc, int32_t bound, const int32_t *nreg0, uint64_t *key, int32_t *par);
int launch_grey_u16(Launch &lc, const void *in, bool u16, uint16_t *out, int32_t n);
int launch_recon_raise(Launch &lc, uint16_t *I, const int32_t *cimg, const uint64_t *key, const int32_t *nreg0,
                       int32_t n);
int launch_wf_compress(Launch &lc, int32_t bound, const int32_t *nreg0, int32_t *par, const int32_t *rlist,
                       int32_t *mlab_k);
int launch_img_counts(Launch &lc, const Img *tab, const Img &one, int32_t nimg, int32_t nl, int32_t ntiles_total,
                      const int32_t *tile_cnt, int64_t *const *outs, int64_t *one_out);

// rag.hip
int launch_rag_gather(Launch &lc, int32_t ntiles, const EdgeSlabs &es, const int32_t *eoff, unsigned long long *keys,
                      int32_t *h);
size_t rag_sort_tmp_bytes(int32_t n);
int rag_sort_reduce(Launch &lc, int32_t n, unsigned long long *keys, int32_t *h, unsigned long long *keys2,
                    int32_t *h2, unsigned long long *ukeys, int32_t *uh, unsigned int *ucount, void *tmp,
                    size_t tmp_bytes);
int launch_rag_final(Launch &lc, const unsigned long long *ukeys, const int32_t *uh, const unsigned int *ucount,
                     const int32_t *rlist, int64_t cap, int32_t *a, int32_t *b, int32_t *hh, int64_t *n_edges);

// gradient.hip
constexpr int FUSED_MAX_R = 16;   // largest blur radius of the fused 2D kernel
int grad_parts(const Geom &g, int ndim, int r);   // partial maxima the magnitude kernels write
int launch_grad_fused2d(Launch &lc, const Geom &g, const float *img, float *mag, float *part, const BlurTaps &taps);
int launch_grad_blur(Launch &lc, const Geom &g, const float *in, float *out, int axis, const BlurTaps &taps);
int launch_grad_sobel(Launch &lc, const Geom &g, int ndim, const float *a, float *mag, float *part);
int launch_grad_max(Launch &lc, int32_t nparts, const float *part, float *tmp, float *gmax);
int launch_grad_quant(Launch &lc, int32_t n, bool u16, const float *mag, void *out, const float *gmax);

}  // namespace wsk
