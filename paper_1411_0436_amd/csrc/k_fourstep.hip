// Two-pass (four-step) spectrometer kernels for 4096 < N <= 2^20: launch
// wrappers around the bodies in fft_bodies.h, for the FP32 and the two
// matrix-core precisions.
#include "fft_bodies.h"

namespace pfbs {

// Minimum waves per SIMD that the column pass's register allocation must
// allow: 4 caps a 512-thread workgroup at 128 VGPRs (two workgroups per CU,
// which their LDS allows).  Measured per sub-FFT length and precision: the
// cap pays where the uncapped kernel needs a little more than 128 registers
// and costs where it forces large spills.
template <int L, int PREC> struct ColsMinWaves {
    static constexpr int value =
        PREC == 0 || (PREC == 1 && L == 128) || (PREC == 2 && (L == 128 || L == 256)) ? 4 : 1;
};

// PT: the pre-filter's tap count as a compile-time constant (its loop fully
// unrolled and software-pipelined), 0 = taken from the arguments.
template <int NPOL, bool PFB, int L, int PREC, int PT = 0>
__global__ __launch_bounds__(kTilePoints / 16 * NPOL, (ColsMinWaves<L, PREC>::value)) void k_front_cols(FrontArgs a) {
    extern __shared__ float smem[];
    front_cols_body<NPOL, PFB, L, PREC, PT>(a, blockIdx.x, gridDim.x, threadIdx.x, smem);
}

template <int NPOL, int L, int PT = 0, int PREC = 0>
__global__ __launch_bounds__(kTilePoints / 16 * NPOL * 2) void k_front_cols_pair(FrontArgs a) {
    extern __shared__ float smem[];
    front_cols_pair_body<NPOL, L, PT, PREC>(a, blockIdx.x, gridDim.x, threadIdx.x, smem);
}


#define PFBS_COLS_CASES(X) X(64) X(128) X(256) X(512)

namespace {
template <int PREC>
hipError_t launch_cols_p(const FrontArgs &a, int npol, bool pfb, dim3 grid, dim3 block, size_t lds,
                         hipStream_t s) {
    switch (a.g.L) {
#define PFBS_PFB(NP, LL)                                                                            \
    switch (pfb ? (a.pt ? a.pt : -1) : 0) {                                                                        \
    case 0: PFBS_LAUNCH((k_front_cols<NP, false, LL, PREC>), grid, block, lds, s, a); break;        \
    case 4: PFBS_LAUNCH((k_front_cols<NP, true, LL, PREC, 4>), grid, block, lds, s, a); break;      \
    case 8: PFBS_LAUNCH((k_front_cols<NP, true, LL, PREC, 8>), grid, block, lds, s, a); break;      \
    default: PFBS_LAUNCH((k_front_cols<NP, true, LL, PREC>), grid, block, lds, s, a); break;        \
    }
#define PFBS_CASE(LL)                                                                               \
    case LL:                                                                                        \
        if (npol == 2) {                                                                            \
            PFBS_PFB(2, LL)                                                                         \
        } else {                                                                                    \
            PFBS_PFB(1, LL)                                                                         \
        }                                                                                           \
        break;
        PFBS_COLS_CASES(PFBS_CASE)
#undef PFBS_CASE
#undef PFBS_PFB
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int PREC>
hipError_t init_fourstep_p(int lds_limit) {
    hipError_t e = hipSuccess;
#define PFBS_ATTR(fn)                                                                            \
    do {                                                                                         \
        hipError_t r = hipFuncSetAttribute(reinterpret_cast<const void *>(fn),                   \
                                           hipFuncAttributeMaxDynamicSharedMemorySize, lds_limit); \
        if (r != hipSuccess) e = r;                                                              \
    } while (0);
#define PFBS_CASE(LL)                              \
    PFBS_ATTR((k_front_cols<2, true, LL, PREC>))   \
    PFBS_ATTR((k_front_cols<2, true, LL, PREC, 4>)) \
    PFBS_ATTR((k_front_cols<2, true, LL, PREC, 8>)) \
    PFBS_ATTR((k_front_cols<2, false, LL, PREC>))  \
    PFBS_ATTR((k_front_cols<1, true, LL, PREC>))   \
    PFBS_ATTR((k_front_cols<1, true, LL, PREC, 4>)) \
    PFBS_ATTR((k_front_cols<1, true, LL, PREC, 8>)) \
    PFBS_ATTR((k_front_cols<1, false, LL, PREC>))
    PFBS_COLS_CASES(PFBS_CASE)
#undef PFBS_CASE
#undef PFBS_ATTR
    return e;
}
}  // namespace

hipError_t launch_front_cols(const FrontArgs &a, int npol, bool pfb, int prec, int n_items, hipStream_t s) {
    const size_t lds = front_lds_bytes(a.g, npol);
    const dim3 grid(n_items * a.ntiles), block(kTilePoints / 16 * npol);
    if (a.pair) {
        if (!pfb || prec < 0 || prec > 2) return hipErrorInvalidValue;
        const dim3 block2(2 * block.x);
        switch (a.g.L) {
#define PFBS_PAIR_P(NP, LL, PR)                                                                          \
    switch (a.pt) {                                                                                      \
    case 4: PFBS_LAUNCH((k_front_cols_pair<NP, LL, 4, PR>), grid, block2, 2 * lds, s, a); break;         \
    case 8: PFBS_LAUNCH((k_front_cols_pair<NP, LL, 8, PR>), grid, block2, 2 * lds, s, a); break;         \
    default: PFBS_LAUNCH((k_front_cols_pair<NP, LL, 0, PR>), grid, block2, 2 * lds, s, a); break;        \
    }
#define PFBS_PAIR(NP, LL)                                                                            \
    if (prec == 0) { PFBS_PAIR_P(NP, LL, 0) }                                                       \
    else if (prec == 1) { PFBS_PAIR_P(NP, LL, 1) }                                                  \
    else { PFBS_PAIR_P(NP, LL, 2) }
#define PFBS_CASE(LL)                                                                                \
    case LL:                                                                                         \
        if (npol == 2) {                                                                             \
            PFBS_PAIR(2, LL)                                                                         \
        } else {                                                                                     \
            PFBS_PAIR(1, LL)                                                                         \
        }                                                                                            \
        break;
            PFBS_COLS_CASES(PFBS_CASE)
#undef PFBS_CASE
#undef PFBS_PAIR
#undef PFBS_PAIR_P
        default:
            return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    switch (prec) {
    case 0: return launch_cols_p<0>(a, npol, pfb, grid, block, lds, s);
    case 1: return launch_cols_p<1>(a, npol, pfb, grid, block, lds, s);
    case 2: return launch_cols_p<2>(a, npol, pfb, grid, block, lds, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_back(const BackArgs &a, int npol, int prec, int n_chunks, hipStream_t s) {
    return prec == 1 || prec == 2 ? launch_back_mfma(a, npol, prec, n_chunks, s)
                                  : launch_back_vector(a, npol, prec, n_chunks, s);
}

hipError_t init_fourstep(int lds_limit) {
    // the row pass: up to 4096-point tiles, FP64 planes (up to 143 KB)
    hipError_t e0 = init_fourstep_p<0>(lds_limit), e1 = init_fourstep_p<1>(lds_limit),
               e2 = init_fourstep_p<2>(lds_limit), e3 = init_back_vector(160 * 1024),
               e4 = init_back_mfma(160 * 1024);
    for (hipError_t e : {e0, e1, e2, e3, e4})
        if (e != hipSuccess) return e;
    return hipSuccess;
}

bool init_fourstep_pair(int lds_limit) {
    bool ok = true;
#define PFBS_PAIR_FNS(LL, PR)                                                                                     \
    reinterpret_cast<const void *>(k_front_cols_pair<2, LL, 0, PR>),                                             \
        reinterpret_cast<const void *>(k_front_cols_pair<2, LL, 4, PR>),                                         \
        reinterpret_cast<const void *>(k_front_cols_pair<2, LL, 8, PR>),                                         \
        reinterpret_cast<const void *>(k_front_cols_pair<1, LL, 0, PR>),                                         \
        reinterpret_cast<const void *>(k_front_cols_pair<1, LL, 4, PR>),                                         \
        reinterpret_cast<const void *>(k_front_cols_pair<1, LL, 8, PR>)
#define PFBS_CASE(LL)                                                                                           \
    for (const void *fn : {PFBS_PAIR_FNS(LL, 0), PFBS_PAIR_FNS(LL, 1), PFBS_PAIR_FNS(LL, 2)})                                \
        if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds_limit) != hipSuccess) ok = false;
    PFBS_COLS_CASES(PFBS_CASE)
#undef PFBS_CASE
#undef PFBS_PAIR_FNS
    (void)hipGetLastError();
    return ok;
}

}  // namespace pfbs
