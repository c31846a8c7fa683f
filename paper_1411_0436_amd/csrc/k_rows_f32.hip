// Row-pass kernels with FP32 and FP64 row arithmetic (see k_rows.h).
#include "k_rows.h"

namespace pfbs {

hipError_t launch_back_vector(const BackArgs &a, int npol, int prec, int n_chunks, hipStream_t s) {
    if (prec == 0) return launch_back_p<0>(a, npol, n_chunks, s);
    if (prec == kRowF64 && a.g.tw64) return launch_back_p<kRowF64>(a, npol, n_chunks, s);
    return hipErrorInvalidValue;
}

hipError_t init_back_vector(int lds_limit) {
    hipError_t e0 = init_back_p<0>(lds_limit), e3 = init_back_p<kRowF64>(lds_limit);
    return e0 != hipSuccess ? e0 : e3;
}

}  // namespace pfbs
