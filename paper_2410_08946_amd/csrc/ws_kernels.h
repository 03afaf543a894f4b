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

// Tiles of one tiling and the launch grid that covers them (one workgroup per
// tile).
struct TileGrid {
    int32_t ntiles = 0;
    int32_t grid = 0;
};

// watershed.hip
#define WS_DECL_SRC(Src)                                                                                          \
    int launch_ws_init(Launch &lc, const Src &src, const TileGrid &tg, int conn, bool u16, int32_t *D,           \
                       int32_t *stamp, int32_t *changed);                                                         \
    int launch_ws_sweep(Launch &lc, const Src &src, const TileGrid &tg, int conn, bool u16, int32_t *D,          \
                        int32_t *stamp, int32_t *changed, int32_t s);                                             \
    int launch_ws_label(Launch &lc, const Src &src, const TileGrid &tg, int conn, bool u16, const int32_t *D,    \
                        int32_t *rec);                                                                            \
    int launch_ws_merge(Launch &lc, const Src &src, const TileGrid &tg, int conn, bool u16, const int32_t *rec); \
    int launch_ws_find(Launch &lc, const Src &src, const TileGrid &tg, int conn);                                \
    int launch_ws_jump(Launch &lc, const Src &src, const TileGrid &tg, int conn, int32_t rr, int32_t *changed);  \
    int launch_wf_init(Launch &lc, const Src &src, const TileGrid &tg, int ndim, int32_t *list, int32_t *count,  \
                       uint64_t *key, int32_t *par, int32_t *tile_tmp, int32_t *tile_cnt0);                       \
    int launch_wf_edge(Launch &lc, const Src &src, const TileGrid &tg, int conn, bool u16, int32_t layer,        \
                       int32_t relabel, const int32_t *par, uint64_t *key, int32_t *tile_cnt);                    \
    int launch_wf_relabel(Launch &lc, const Src &src, const TileGrid &tg, int ndim, int32_t layer,               \
                          const int32_t *par, int32_t *tile_cnt);
WS_DECL_SRC(OneImg)
WS_DECL_SRC(ImgTable)
#undef WS_DECL_SRC

int border_cells(int ndim);
int launch_ws_stages(Launch &lc, const Geom &g, int conn, bool u16, const void *I, const int32_t *D, int32_t *bal,
                     int32_t *arrow);
int launch_fill_i32(Launch &lc, int32_t *a, int32_t n, int32_t v);

// waterfall.hip
int compact_chunks(int32_t bound);
int wf_tiles(const Geom &g, int ndim);
int launch_wf_union(Launch &lc, int32_t bound, const int32_t *list, const int32_t *count, uint64_t *key, int32_t *par);
int launch_wf_compress(Launch &lc, int32_t bound, const int32_t *list, const int32_t *count, int32_t *par);
int launch_wf_compact(Launch &lc, int32_t bound, const int32_t *list_in, const int32_t *count_in, int32_t *list_out,
                      int32_t *count_out, const int32_t *par, uint64_t *key, int32_t *chunk_tmp);
int launch_img_counts(Launch &lc, const Img *tab, const Img &one, int32_t nimg, int32_t nl, int32_t ntiles_total,
                      const int32_t *tile_cnt, int64_t *const *outs, int64_t *one_out);

// gradient.hip
constexpr int FUSED_MAX_R = 16;   // largest blur radius of the fused 2D kernel
int launch_grad_fused2d(Launch &lc, const Geom &g, const float *img, float *mag, unsigned int *slots, const BlurTaps &taps);
int launch_grad_blur(Launch &lc, const Geom &g, const float *in, float *out, int axis, const BlurTaps &taps);
int launch_grad_sobel(Launch &lc, const Geom &g, int ndim, const float *a, float *mag, unsigned int *slots);
int launch_grad_quant(Launch &lc, int32_t n, bool u16, const float *mag, void *out, const unsigned int *slots);
int launch_grad_zero_slots(Launch &lc, unsigned int *slots);

}  // namespace wsk
