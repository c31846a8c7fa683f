// Two-pass (four-step) spectrometer kernels for 4096 < N <= 2^20: launch
// wrappers around the bodies in fft_bodies.h.
#include "fft_bodies.h"

namespace pfbs {

template <int NPOL, bool PFB, int L>
__global__ __launch_bounds__(kTilePoints / 16 * NPOL) void k_front_cols(FrontArgs a) {
    front_cols_body<NPOL, PFB, L>(a, blockIdx.x, gridDim.x);
}

template <int NPOL, int L>
__global__ __launch_bounds__(BackTile<L>::TP / 16 * NPOL) void k_back(BackArgs a) {
    back_body<NPOL, L>(a, blockIdx.x);
}

#define PFBS_COLS_CASES(X) X(64) X(128) X(256) X(512)
#define PFBS_BACK_CASES(X) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096)

hipError_t launch_front_cols(const FrontArgs &a, int npol, bool pfb, int n_items, hipStream_t s) {
    const size_t lds = front_lds_bytes(a.g, npol);
    const dim3 grid(n_items * a.ntiles), block(kTilePoints / 16 * npol);
    switch (a.g.L) {
#define PFBS_CASE(LL)                                                                           \
    case LL:                                                                                    \
        if (npol == 2) {                                                                        \
            if (pfb) hipLaunchKernelGGL((k_front_cols<2, true, LL>), grid, block, lds, s, a);   \
            else hipLaunchKernelGGL((k_front_cols<2, false, LL>), grid, block, lds, s, a);      \
        } else {                                                                                \
            if (pfb) hipLaunchKernelGGL((k_front_cols<1, true, LL>), grid, block, lds, s, a);   \
            else hipLaunchKernelGGL((k_front_cols<1, false, LL>), grid, block, lds, s, a);      \
        }                                                                                       \
        break;
        PFBS_COLS_CASES(PFBS_CASE)
#undef PFBS_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_back(const BackArgs &a, int npol, int n_chunks, hipStream_t s) {
    const size_t lds = back_lds_bytes(a.g, npol);
    const dim3 grid(n_chunks * a.ntiles), block(a.g.T * a.g.L / 16 * npol);
    switch (a.g.L) {
#define PFBS_CASE(LL)                                                              \
    case LL:                                                                       \
        if (npol == 2) hipLaunchKernelGGL((k_back<2, LL>), grid, block, lds, s, a); \
        else hipLaunchKernelGGL((k_back<1, LL>), grid, block, lds, s, a);           \
        break;
        PFBS_BACK_CASES(PFBS_CASE)
#undef PFBS_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t init_fourstep(int lds_limit) {
    hipError_t e = hipSuccess;
#define PFBS_ATTR(fn)                                                                            \
    do {                                                                                         \
        hipError_t r = hipFuncSetAttribute(reinterpret_cast<const void *>(fn),                   \
                                           hipFuncAttributeMaxDynamicSharedMemorySize, lds_limit); \
        if (r != hipSuccess) e = r;                                                              \
    } while (0);
#define PFBS_CASE(LL)                        \
    PFBS_ATTR((k_front_cols<2, true, LL>))   \
    PFBS_ATTR((k_front_cols<2, false, LL>))  \
    PFBS_ATTR((k_front_cols<1, true, LL>))   \
    PFBS_ATTR((k_front_cols<1, false, LL>))
    PFBS_COLS_CASES(PFBS_CASE)
#undef PFBS_CASE
#define PFBS_CASE(LL) PFBS_ATTR((k_back<2, LL>)) PFBS_ATTR((k_back<1, LL>))
    PFBS_BACK_CASES(PFBS_CASE)
#undef PFBS_CASE
#undef PFBS_ATTR
    return e;
}

}  // namespace pfbs
