// Row-pass kernels on the matrix cores: FP16 and split-FP16 DFT-16 stages
// (see k_rows.h).
#include "k_rows.h"

namespace pfbs {

hipError_t launch_back_mfma(const BackArgs &a, int npol, int prec, int n_chunks, hipStream_t s) {
    if (prec == 1) return launch_back_p<1>(a, npol, n_chunks, s);
    if (prec == 2) return launch_back_p<2>(a, npol, n_chunks, s);
    return hipErrorInvalidValue;
}

hipError_t init_back_mfma(int lds_limit) {
    hipError_t e1 = init_back_p<1>(lds_limit), e2 = init_back_p<2>(lds_limit);
    return e1 != hipSuccess ? e1 : e2;
}

}  // namespace pfbs
