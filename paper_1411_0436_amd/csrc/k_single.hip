// Single-pass spectrometer kernel for N <= 4096: launch wrappers around the
// body in fft_bodies.h, for the FP32 and the two matrix-core precisions.
#include "fft_bodies.h"

namespace pfbs {

// PT: the pre-filter's tap count as a compile-time constant (its loop fully
// unrolled and software-pipelined), 0 = taken from the arguments.
template <int NPOL, bool PFB, int L, int PREC, int PT = 0>
__global__ __launch_bounds__(kTilePoints / 16 * NPOL) void k_front_single(FrontArgs a) {
    extern __shared__ float smem[];
    front_single_body<NPOL, PFB, L, PREC, PT>(a, blockIdx.x, threadIdx.x, smem);
}

#define PFBS_SINGLE_CASES(X) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096)

namespace {
template <int PREC>
hipError_t launch_single_p(const FrontArgs &a, int npol, bool pfb, dim3 grid, dim3 block, size_t lds,
                           hipStream_t s) {
    switch (a.g.L) {
#define PFBS_PFB(NP, LL)                                                                              \
    switch (pfb ? (a.pt ? a.pt : -1) : 0) {                                                                          \
    case 0: PFBS_LAUNCH((k_front_single<NP, false, LL, PREC>), grid, block, lds, s, a); break;        \
    case 4: PFBS_LAUNCH((k_front_single<NP, true, LL, PREC, 4>), grid, block, lds, s, a); break;      \
    case 8: PFBS_LAUNCH((k_front_single<NP, true, LL, PREC, 8>), grid, block, lds, s, a); break;      \
    default: PFBS_LAUNCH((k_front_single<NP, true, LL, PREC>), grid, block, lds, s, a); break;        \
    }
#define PFBS_CASE(LL)                                                                                 \
    case LL:                                                                                          \
        if (npol == 2) {                                                                              \
            PFBS_PFB(2, LL)                                                                           \
        } else {                                                                                      \
            PFBS_PFB(1, LL)                                                                           \
        }                                                                                             \
        break;
        PFBS_SINGLE_CASES(PFBS_CASE)
#undef PFBS_CASE
#undef PFBS_PFB
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int PREC>
hipError_t init_single_p(int lds_limit) {
    hipError_t e = hipSuccess;
#define PFBS_ATTR(fn)                                                                            \
    do {                                                                                         \
        hipError_t r = hipFuncSetAttribute(reinterpret_cast<const void *>(fn),                   \
                                           hipFuncAttributeMaxDynamicSharedMemorySize, lds_limit); \
        if (r != hipSuccess) e = r;                                                              \
    } while (0);
#define PFBS_CASE(LL)                                \
    PFBS_ATTR((k_front_single<2, true, LL, PREC>))   \
    PFBS_ATTR((k_front_single<2, true, LL, PREC, 4>)) \
    PFBS_ATTR((k_front_single<2, true, LL, PREC, 8>)) \
    PFBS_ATTR((k_front_single<2, false, LL, PREC>))  \
    PFBS_ATTR((k_front_single<1, true, LL, PREC>))   \
    PFBS_ATTR((k_front_single<1, true, LL, PREC, 4>)) \
    PFBS_ATTR((k_front_single<1, true, LL, PREC, 8>)) \
    PFBS_ATTR((k_front_single<1, false, LL, PREC>))
    PFBS_SINGLE_CASES(PFBS_CASE)
#undef PFBS_CASE
#undef PFBS_ATTR
    return e;
}
}  // namespace

hipError_t launch_front_single(const FrontArgs &a, int npol, bool pfb, int prec, int n_chunks,
                               hipStream_t s) {
    const size_t lds = front_lds_bytes(a.g, npol);
    const dim3 grid(n_chunks), block(kTilePoints / 16 * npol);
    switch (prec) {
    case 0: return launch_single_p<0>(a, npol, pfb, grid, block, lds, s);
    case 1: return launch_single_p<1>(a, npol, pfb, grid, block, lds, s);
    case 2: return launch_single_p<2>(a, npol, pfb, grid, block, lds, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t init_single(int lds_limit) {
    hipError_t e0 = init_single_p<0>(lds_limit), e1 = init_single_p<1>(lds_limit),
               e2 = init_single_p<2>(lds_limit);
    return e0 != hipSuccess ? e0 : (e1 != hipSuccess ? e1 : e2);
}

}  // namespace pfbs
