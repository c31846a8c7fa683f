// Batched launches for several sub-bands.  Entries of one kernel variant
// (kind, polarisations, filter, sub-FFT length) share one launch; each
// workgroup finds its sub-band entry from its block id and runs the same
// device body as that sub-band's own kernel, at that kernel's own register
// budget.  The paper's eight-sub-band mode runs its 16 FFTs in parallel
// (Section 4) and attributes small-N slowness to per-batch launch overhead
// (Section 5); here a block of all sub-bands is a handful of launches, which
// can be replayed from one HIP graph.
#include "fft_bodies.h"

namespace pfbs {

template <class E>
__device__ __forceinline__ int find_entry(const E *t, int n, int bid) {
    int e = 0;
    while (e + 1 < n && bid >= t[e + 1].wg0) ++e;
    return e;
}

template <int NPOL, bool PFB, int L, int PT = 0>
__global__ __launch_bounds__(kTilePoints / 16 * NPOL) void k_multi_single(const BatchFrontEntry *__restrict__ t, int n) {
    if (n <= 0) return;
    const int e = find_entry(t, n, blockIdx.x);
    const int vb = blockIdx.x - t[e].wg0;
    if (vb < 0 || vb >= t[e].wgn) return;
    // a private copy: the body's global stores cannot alias it, so its fields
    // stay in registers instead of being reloaded after every store
    FrontArgs a = t[e].a;
    globalise(a);
    front_single_body<NPOL, PFB, L, 0, PT>(a, vb);
}

template <int NPOL, bool PFB, int L, int PT = 0>
__global__ __launch_bounds__(kTilePoints / 16 * NPOL) void k_multi_cols(const BatchFrontEntry *__restrict__ t, int n) {
    if (n <= 0) return;
    const int e = find_entry(t, n, blockIdx.x);
    const int vb = blockIdx.x - t[e].wg0, wgn = t[e].wgn;
    if (vb < 0 || vb >= wgn) return;
    FrontArgs a = t[e].a;
    globalise(a);
    front_cols_body<NPOL, PFB, L, 0, PT>(a, vb, wgn);
}

template <int NPOL, int L, int PREC = 0>
__global__ __launch_bounds__(BackTile<L>::TP / 16 * NPOL) void k_multi_back(const BatchBackEntry *__restrict__ t, int n) {
    if (n <= 0) return;
    const int e = find_entry(t, n, blockIdx.x);
    const int vb = blockIdx.x - t[e].wg0;
    if (vb < 0 || vb >= t[e].wgn) return;
    BackArgs a = t[e].a;
    globalise(a);
    back_body<NPOL, L, PREC>(a, vb);
}

#define PFBS_M_SINGLE(X) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096)
#define PFBS_M_COLS(X) X(64) X(128) X(256) X(512)
#define PFBS_M_BACK(X) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096)

// pt: compile-time tap count of the variant (4 or 8), 0 = from the entry.
const void *multi_front_fn(int npol, int kind, int pfb, int L, int pt) {
#define PFBS_F(KERN, LL)                                                                       \
    if (L == LL) {                                                                             \
        if (npol == 2) {                                                                       \
            if (!pfb) return reinterpret_cast<const void *>(&KERN<2, false, LL>);              \
            if (pt == 4) return reinterpret_cast<const void *>(&KERN<2, true, LL, 4>);         \
            if (pt == 8) return reinterpret_cast<const void *>(&KERN<2, true, LL, 8>);         \
            return reinterpret_cast<const void *>(&KERN<2, true, LL>);                         \
        }                                                                                      \
        if (!pfb) return reinterpret_cast<const void *>(&KERN<1, false, LL>);                  \
        if (pt == 4) return reinterpret_cast<const void *>(&KERN<1, true, LL, 4>);             \
        if (pt == 8) return reinterpret_cast<const void *>(&KERN<1, true, LL, 8>);             \
        return reinterpret_cast<const void *>(&KERN<1, true, LL>);                             \
    }
    if (kind == 0) {
#define PFBS_S(LL) PFBS_F(k_multi_single, LL)
        PFBS_M_SINGLE(PFBS_S)
#undef PFBS_S
    } else {
#define PFBS_C(LL) PFBS_F(k_multi_cols, LL)
        PFBS_M_COLS(PFBS_C)
#undef PFBS_C
    }
#undef PFBS_F
    return nullptr;
}

// prec: 0 FP32, 3 FP64 row pass.
const void *multi_back_fn(int npol, int L, int prec) {
#define PFBS_B(LL)                                                                                   \
    if (L == LL) {                                                                                   \
        if (prec == 3) return npol == 2 ? reinterpret_cast<const void *>(&k_multi_back<2, LL, 3>)    \
                                        : reinterpret_cast<const void *>(&k_multi_back<1, LL, 3>);   \
        if (prec == 0) return npol == 2 ? reinterpret_cast<const void *>(&k_multi_back<2, LL>)       \
                                        : reinterpret_cast<const void *>(&k_multi_back<1, LL>);      \
    }
    PFBS_M_BACK(PFBS_B)
#undef PFBS_B
    return nullptr;
}

hipError_t init_batch(int lds_limit) {
    hipError_t e = hipSuccess;
    for (int npol = 1; npol <= 2; ++npol)
        for (int pfb = 0; pfb <= 1; ++pfb)
            for (int kind = 0; kind <= 1; ++kind)
                for (int L = 16; L <= 4096; L *= 2)
                    for (int pt : {0, 4, 8}) {
                        const void *f = multi_front_fn(npol, kind, pfb, L, pt);
                        if (!f) continue;
                        hipError_t r = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds_limit);
                        if (r != hipSuccess) e = r;
                    }
    for (int npol = 1; npol <= 2; ++npol)
        for (int L = 32; L <= 4096; L *= 2)
            for (int prec : {0, 3}) {
                const void *f = multi_back_fn(npol, L, prec);
                if (!f) continue;
                hipError_t r = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds_limit);
                if (r != hipSuccess) e = r;
            }
    return e;
}

}  // namespace pfbs
