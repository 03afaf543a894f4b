// rag.hip -- region adjacency graph export: the distinct pairs of adjacent
// regions of one labelling with their lowest boundary pass, the graph on which
// the waterfall's layers are built (Section 4; the regions and their pass
// heights are what downstream superpixel graph models consume).
//
// The waterfall's pixel pass leaves every tile's distinct edges (region ids,
// lowest height within the tile) in its slab. Here the slabs are gathered into
// one list of 64-bit keys (id_a << 32 | id_b, id_a < id_b) with heights, sorted
// (device radix sort), and equal keys are reduced to their lowest height;
// region ids are in label order, so the result is sorted by (label a, label b).
#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_reduce_by_key.hpp>

#include "ws_device.h"
#include "ws_kernels.h"

namespace wsk {

// Edges of tile t (ecnt[t] of them, at t * cap in the slabs) to eoff[t] ...
__global__ __launch_bounds__(NTHREADS) void k_rag_gather(int32_t ntiles, int32_t cap, const uint64_t *__restrict__ ep,
                                                         const uint16_t *__restrict__ ew,
                                                         const int32_t *__restrict__ ecnt,
                                                         const int32_t *__restrict__ eoff,
                                                         unsigned long long *__restrict__ keys,
                                                         int32_t *__restrict__ h) {
    const int t = blockIdx.x;
    if (t >= ntiles) return;
    const int32_t n = ecnt[t], o = eoff[t];
    const size_t base = (size_t)t * (size_t)cap;
    for (int32_t i = threadIdx.x; i < n; i += NTHREADS) {
        keys[o + i] = (unsigned long long)ep[base + i];
        h[o + i] = (int32_t)ew[base + i];
    }
}

// Unique edges (ids) -> labels; at most cap written; *n_edges = their number.
__global__ __launch_bounds__(NTHREADS) void k_rag_final(const unsigned long long *__restrict__ ukeys,
                                                        const int32_t *__restrict__ uh,
                                                        const unsigned int *__restrict__ ucount,
                                                        const int32_t *__restrict__ rlist, int64_t cap,
                                                        int32_t *__restrict__ a, int32_t *__restrict__ b,
                                                        int32_t *__restrict__ hh, int64_t *__restrict__ n_edges) {
    const int64_t n = *ucount;
    if (blockIdx.x == 0 && threadIdx.x == 0 && n_edges) *n_edges = n;
    const int64_t m = n < cap ? n : cap;
    for (int64_t i = (int64_t)blockIdx.x * NTHREADS + threadIdx.x; i < m; i += (int64_t)gridDim.x * NTHREADS) {
        unsigned long long k = ukeys[i];
        a[i] = rlist[(int32_t)(k >> 32)];
        b[i] = rlist[(int32_t)(uint32_t)k];
        hh[i] = uh[i];
    }
}

int launch_rag_gather(Launch &lc, int32_t ntiles, const EdgeSlabs &es, const int32_t *eoff, unsigned long long *keys,
                      int32_t *h) {
    return lc.run("rag", k_rag_gather, dim3(ntiles > 0 ? ntiles : 1), dim3(NTHREADS), ntiles, es.cap,
                  (const uint64_t *)es.p, (const uint16_t *)es.w, (const int32_t *)es.cnt, eoff, keys, h);
}

size_t rag_sort_tmp_bytes(int32_t n) {
    size_t a = 0, b = 0;
    (void)rocprim::radix_sort_pairs(nullptr, a, (unsigned long long *)nullptr, (unsigned long long *)nullptr,
                                    (int32_t *)nullptr, (int32_t *)nullptr, (size_t)n, 0, 64);
    (void)rocprim::reduce_by_key(nullptr, b, (unsigned long long *)nullptr, (int32_t *)nullptr, (size_t)n,
                                 (unsigned long long *)nullptr, (int32_t *)nullptr, (unsigned int *)nullptr,
                                 rocprim::minimum<int32_t>(), rocprim::equal_to<unsigned long long>());
    return (a > b ? a : b) + 256;
}

int rag_sort_reduce(Launch &lc, int32_t n, unsigned long long *keys, int32_t *h, unsigned long long *keys2,
                    int32_t *h2, unsigned long long *ukeys, int32_t *uh, unsigned int *ucount, void *tmp,
                    size_t tmp_bytes) {
    size_t tb = tmp_bytes;
    hipError_t e = rocprim::radix_sort_pairs(tmp, tb, keys, keys2, h, h2, (size_t)n, 0, 64, lc.stream);
    if (e != hipSuccess) {
        lc.last = e;
        return -3;
    }
    tb = tmp_bytes;
    e = rocprim::reduce_by_key(tmp, tb, keys2, h2, (size_t)n, ukeys, uh, ucount, rocprim::minimum<int32_t>(),
                               rocprim::equal_to<unsigned long long>(), lc.stream);
    if (e != hipSuccess) {
        lc.last = e;
        return -3;
    }
    return 0;
}

int launch_rag_final(Launch &lc, const unsigned long long *ukeys, const int32_t *uh, const unsigned int *ucount,
                     const int32_t *rlist, int64_t cap, int32_t *a, int32_t *b, int32_t *hh, int64_t *n_edges) {
    int64_t blocks = (cap + NTHREADS - 1) / NTHREADS;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    return lc.run("rag", k_rag_final, dim3((uint32_t)blocks), dim3(NTHREADS), ukeys, uh, ucount, rlist, cap, a, b, hh,
                  n_edges);
}

}  // namespace wsk
