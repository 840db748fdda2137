// Streaming probes: the attainable HBM bandwidth that the stencil passes are compared with.
// Three access patterns over device arrays, 16 bytes per lane per step (one double2), a
// grid-stride loop over a fixed grid of a few blocks per compute unit:
//   read  - every element of a is loaded and summed (one partial per block is stored, so
//           the loads cannot be dropped);
//   copy  - c = a;
//   triad - c = a + b (two streams in, one out: the shape of a smoothing pass, which reads
//           u and f and writes u).
// Stores are non-temporal, as in the passes.  fas_stream_probe times `reps` launches with
// HIP events recorded on the caller's stream and reports the average duration.
#include <hip/hip_runtime.h>

#include "fas_device.h"
#include "fas_internal.h"

namespace fas {

namespace {

constexpr int kStreamBlock = 256;

template <int KIND>
__global__ __launch_bounds__(kStreamBlock) void k_stream(int64_t n2, const double2* __restrict__ a,
                                                         const double2* __restrict__ b, double2* __restrict__ c,
                                                         double* __restrict__ part)
{
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kStreamBlock;
    for (int64_t i = (int64_t)blockIdx.x * kStreamBlock + threadIdx.x; i < n2; i += stride) {
        const double2 x = a[i];
        if constexpr (KIND == 0) {
            acc += x.x + x.y;
        } else if constexpr (KIND == 1) {
            store_pair_nt(reinterpret_cast<double*>(c + i), x.x, x.y);
        } else {
            const double2 y = b[i];
            store_pair_nt(reinterpret_cast<double*>(c + i), x.x + y.x, x.y + y.y);
        }
    }
    if constexpr (KIND == 0) {
        __shared__ double red[kStreamBlock];
        red[threadIdx.x] = acc;
        __syncthreads();
        for (int s = kStreamBlock / 2; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[blockIdx.x] = red[0];
    }
}

}  // namespace

}  // namespace fas

extern "C" int fas_stream_probe(void* stream, int kind, int64_t bytes, const void* a, const void* b, void* c,
                                double* part, int blocks, int reps, double* ms_out)
{
    using namespace fas;
    if (kind < 0 || kind > 2 || bytes <= 0 || bytes % 16 || !a || reps < 1 || blocks < 1 || !ms_out) return FAS_ERR_ARG;
    if ((kind == 0 && !part) || (kind >= 1 && !c) || (kind == 2 && !b)) return FAS_ERR_ARG;
    if (((uintptr_t)a | (uintptr_t)b | (uintptr_t)c) % 16) return FAS_ERR_ARG;
    const hipStream_t s = (hipStream_t)stream;
    const int64_t n2 = bytes / 16;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return FAS_ERR_HIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return FAS_ERR_HIP;
    }
    auto launch = [&]() {
        const auto A = (const double2*)a;
        const auto B = (const double2*)b;
        const auto C = (double2*)c;
        if (kind == 0)
            k_stream<0><<<blocks, kStreamBlock, 0, s>>>(n2, A, B, C, part);
        else if (kind == 1)
            k_stream<1><<<blocks, kStreamBlock, 0, s>>>(n2, A, B, C, part);
        else
            k_stream<2><<<blocks, kStreamBlock, 0, s>>>(n2, A, B, C, part);
    };
    launch();  // warm-up
    int rc = FAS_OK;
    if (hipEventRecord(e0, s) != hipSuccess) rc = FAS_ERR_HIP;
    for (int r = 0; r < reps && rc == FAS_OK; ++r) launch();
    if (rc == FAS_OK && hipGetLastError() != hipSuccess) rc = FAS_ERR_HIP;
    if (rc == FAS_OK && hipEventRecord(e1, s) != hipSuccess) rc = FAS_ERR_HIP;
    if (rc == FAS_OK && hipEventSynchronize(e1) != hipSuccess) rc = FAS_ERR_HIP;
    float ms = 0.f;
    if (rc == FAS_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = FAS_ERR_HIP;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == FAS_OK) *ms_out = ms / reps;
    return rc;
}
