// Row pass of the two-pass FFT (outer sub-FFTs, polarisation products and
// their accumulation): kernel wrappers around back_body for every row length
// L and tile size TP (points per polarisation per workgroup step, TP / L rows
// per step: the workgroup has TP / 16 threads per polarisation).  The plan's
// default tile is BackTile<L>::TP; larger tiles are a tuning choice.  Each
// precision's kernels are built in a translation unit of their own
// (k_rows_f32.hip: FP32 and FP64 row arithmetic; k_rows_mfma.hip: the
// matrix-core precisions).
#pragma once

#include "fft_bodies.h"

namespace pfbs {

template <int NPOL, int L, int PREC, int TP>
__global__ __launch_bounds__(TP / 16 * NPOL) void k_back(BackArgs a) {
    extern __shared__ float smem[];
    back_body<NPOL, L, PREC, TP>(a, blockIdx.x, threadIdx.x, smem);
}

#define PFBS_ROW_LENGTHS(X) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096)

// Every (L, TP) with TP in {1024, 2048, 4096} and TP >= max(L, 1024).
template <int PREC, class F>
void for_each_row_kernel(F &&f) {
#define PFBS_ROW_TP(NP, LL, TP) \
    if constexpr (TP >= LL) f(NP, LL, TP, reinterpret_cast<const void *>(&k_back<NP, LL, PREC, TP>));
#define PFBS_ROW_L(LL)                                                                            \
    PFBS_ROW_TP(2, LL, 1024) PFBS_ROW_TP(2, LL, 2048) PFBS_ROW_TP(2, LL, 4096)                    \
    PFBS_ROW_TP(1, LL, 1024) PFBS_ROW_TP(1, LL, 2048) PFBS_ROW_TP(1, LL, 4096)
    PFBS_ROW_LENGTHS(PFBS_ROW_L)
#undef PFBS_ROW_L
#undef PFBS_ROW_TP
}

template <int PREC>
hipError_t launch_back_p(const BackArgs &a, int npol, int n_chunks, hipStream_t s) {
    const int L = a.g.L, TP = a.g.T * a.g.L;
    const void *fn = nullptr;
    for_each_row_kernel<PREC>([&](int np, int l, int tp, const void *k) {
        if (np == npol && l == L && tp == TP) fn = k;
    });
    if (!fn) return hipErrorInvalidValue;
    const size_t lds = back_lds_bytes(a.g, npol, PREC);
    const dim3 grid(n_chunks * a.ntiles), block(TP / 16 * npol);
    BackArgs arg = a;
    void *args[] = {&arg};
    if (g_launch_events.start)
        return hipExtLaunchKernel(fn, grid, block, args, lds, s, g_launch_events.start, g_launch_events.stop, 0);
    return hipLaunchKernel(fn, grid, block, args, lds, s);
}

template <int PREC>
hipError_t init_back_p(int lds_limit) {
    hipError_t e = hipSuccess;
    for_each_row_kernel<PREC>([&](int, int, int, const void *k) {
        hipError_t r = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lds_limit);
        if (r != hipSuccess) e = r;
    });
    return e;
}

}  // namespace pfbs
