// Single-pass spectrometer kernel for N <= 4096: launch wrappers around the
// body in fft_bodies.h.
#include "fft_bodies.h"

namespace pfbs {

template <int NPOL, bool PFB, int L>
__global__ __launch_bounds__(kTilePoints / 16 * NPOL) void k_front_single(FrontArgs a) {
    front_single_body<NPOL, PFB, L>(a, blockIdx.x);
}

#define PFBS_SINGLE_CASES(X) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096)

hipError_t launch_front_single(const FrontArgs &a, int npol, bool pfb, int n_chunks, hipStream_t s) {
    const size_t lds = front_lds_bytes(a.g, npol);
    const dim3 grid(n_chunks), block(kTilePoints / 16 * npol);
    switch (a.g.L) {
#define PFBS_CASE(LL)                                                                              \
    case LL:                                                                                       \
        if (npol == 2) {                                                                           \
            if (pfb) hipLaunchKernelGGL((k_front_single<2, true, LL>), grid, block, lds, s, a);    \
            else hipLaunchKernelGGL((k_front_single<2, false, LL>), grid, block, lds, s, a);       \
        } else {                                                                                   \
            if (pfb) hipLaunchKernelGGL((k_front_single<1, true, LL>), grid, block, lds, s, a);    \
            else hipLaunchKernelGGL((k_front_single<1, false, LL>), grid, block, lds, s, a);       \
        }                                                                                          \
        break;
        PFBS_SINGLE_CASES(PFBS_CASE)
#undef PFBS_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t init_single(int lds_limit) {
    hipError_t e = hipSuccess;
#define PFBS_ATTR(fn)                                                                            \
    do {                                                                                         \
        hipError_t r = hipFuncSetAttribute(reinterpret_cast<const void *>(fn),                   \
                                           hipFuncAttributeMaxDynamicSharedMemorySize, lds_limit); \
        if (r != hipSuccess) e = r;                                                              \
    } while (0);
#define PFBS_CASE(LL)                          \
    PFBS_ATTR((k_front_single<2, true, LL>))   \
    PFBS_ATTR((k_front_single<2, false, LL>))  \
    PFBS_ATTR((k_front_single<1, true, LL>))   \
    PFBS_ATTR((k_front_single<1, false, LL>))
    PFBS_SINGLE_CASES(PFBS_CASE)
#undef PFBS_CASE
#undef PFBS_ATTR
    return e;
}

}  // namespace pfbs
