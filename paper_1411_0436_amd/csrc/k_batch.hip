// Batched dispatcher kernels: one launch per phase for every sub-band of a
// batch (the paper's eight-sub-band mode runs its 16 FFTs in parallel,
// Section 4, and attributes small-N slowness to per-batch launch overhead,
// Section 5).  Each workgroup finds its sub-band entry from its block id and
// runs the same device body as the sub-band's own kernel would.
#include "fft_bodies.h"

namespace pfbs {

template <class E>
__device__ __forceinline__ int find_entry(const E *t, int n, int bid) {
    int e = 0;
    while (e + 1 < n && bid >= t[e + 1].wg0) ++e;
    return e;
}

#define PFBS_FRONT_SINGLE(X) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096)
#define PFBS_FRONT_COLS(X) X(64) X(128) X(256) X(512)

template <int NPOL>
__global__ __launch_bounds__(kTilePoints / 16 * NPOL) void k_batch_front(const BatchFrontEntry *t, int n) {
    if (n <= 0) return;
    const int e = find_entry(t, n, blockIdx.x);
    const BatchFrontEntry &E = t[e];
    const int vb = blockIdx.x - E.wg0;
    if (vb < 0 || vb >= E.wgn) return;
    if (E.kind == 0) {
        switch (E.L) {
#define PFBS_C(LL)                                                              \
    case LL:                                                                    \
        if (E.pfb) front_single_body<NPOL, true, LL>(E.a, vb);                  \
        else front_single_body<NPOL, false, LL>(E.a, vb);                       \
        break;
            PFBS_FRONT_SINGLE(PFBS_C)
#undef PFBS_C
        default:
            break;
        }
    } else {
        switch (E.L) {
#define PFBS_C(LL)                                                              \
    case LL:                                                                    \
        if (E.pfb) front_cols_body<NPOL, true, LL>(E.a, vb, E.wgn);             \
        else front_cols_body<NPOL, false, LL>(E.a, vb, E.wgn);                  \
        break;
            PFBS_FRONT_COLS(PFBS_C)
#undef PFBS_C
        default:
            break;
        }
    }
}

// Row-pass bodies grouped by workgroup size: rows up to 1024 points use 64
// threads per polarisation, 2048 and 4096 use 128 and 256.
template <int NPOL, int TPP>
__global__ __launch_bounds__(TPP *NPOL) void k_batch_back(const BatchBackEntry *t, int n) {
    if (n <= 0) return;
    const int e = find_entry(t, n, blockIdx.x);
    const BatchBackEntry &E = t[e];
    const int vb = blockIdx.x - E.wg0;
    if (vb < 0 || vb >= E.wgn) return;
    if constexpr (TPP == 64) {
        switch (E.L) {
        case 32: back_body<NPOL, 32>(E.a, vb); break;
        case 64: back_body<NPOL, 64>(E.a, vb); break;
        case 128: back_body<NPOL, 128>(E.a, vb); break;
        case 256: back_body<NPOL, 256>(E.a, vb); break;
        case 512: back_body<NPOL, 512>(E.a, vb); break;
        case 1024: back_body<NPOL, 1024>(E.a, vb); break;
        default: break;
        }
    } else if constexpr (TPP == 128) {
        if (E.L == 2048) back_body<NPOL, 2048>(E.a, vb);
    } else {
        if (E.L == 4096) back_body<NPOL, 4096>(E.a, vb);
    }
}

hipError_t launch_batch_front(const BatchFrontEntry *t, int n, int total_wg, int npol, size_t lds,
                              hipStream_t s) {
    const dim3 grid(total_wg > 0 ? total_wg : 1), block(kTilePoints / 16 * npol);
    if (npol == 2) hipLaunchKernelGGL((k_batch_front<2>), grid, block, lds, s, t, n);
    else hipLaunchKernelGGL((k_batch_front<1>), grid, block, lds, s, t, n);
    return hipGetLastError();
}

hipError_t launch_batch_back(const BatchBackEntry *t, int n, int total_wg, int npol, int threads,
                             size_t lds, hipStream_t s) {
    const dim3 grid(total_wg > 0 ? total_wg : 1), block(threads);
    const int tpp = threads / npol;
    if (npol == 2) {
        if (tpp == 64) hipLaunchKernelGGL((k_batch_back<2, 64>), grid, block, lds, s, t, n);
        else if (tpp == 128) hipLaunchKernelGGL((k_batch_back<2, 128>), grid, block, lds, s, t, n);
        else hipLaunchKernelGGL((k_batch_back<2, 256>), grid, block, lds, s, t, n);
    } else {
        if (tpp == 64) hipLaunchKernelGGL((k_batch_back<1, 64>), grid, block, lds, s, t, n);
        else if (tpp == 128) hipLaunchKernelGGL((k_batch_back<1, 128>), grid, block, lds, s, t, n);
        else hipLaunchKernelGGL((k_batch_back<1, 256>), grid, block, lds, s, t, n);
    }
    return hipGetLastError();
}

const void *batch_front_fn(int npol) {
    return npol == 2 ? reinterpret_cast<const void *>(&k_batch_front<2>)
                     : reinterpret_cast<const void *>(&k_batch_front<1>);
}

const void *batch_back_fn(int npol, int threads) {
    const int tpp = threads / npol;
    if (npol == 2) {
        if (tpp == 64) return reinterpret_cast<const void *>(&k_batch_back<2, 64>);
        if (tpp == 128) return reinterpret_cast<const void *>(&k_batch_back<2, 128>);
        return reinterpret_cast<const void *>(&k_batch_back<2, 256>);
    }
    if (tpp == 64) return reinterpret_cast<const void *>(&k_batch_back<1, 64>);
    if (tpp == 128) return reinterpret_cast<const void *>(&k_batch_back<1, 128>);
    return reinterpret_cast<const void *>(&k_batch_back<1, 256>);
}

size_t back_lds_bytes_for(int L, int npol) {
    Geo g;
    g.L = L;
    g.T = (L < 1024 ? 1024 : L) / L;
    g.tw = nullptr;
    return back_lds_bytes(g, npol);
}

hipError_t init_batch(int lds_limit) {
    hipError_t e = hipSuccess;
    const void *fns[] = {batch_front_fn(2), batch_front_fn(1), batch_back_fn(2, 128), batch_back_fn(2, 256),
                         batch_back_fn(2, 512), batch_back_fn(1, 64), batch_back_fn(1, 128),
                         batch_back_fn(1, 256)};
    for (const void *f : fns) {
        hipError_t r = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds_limit);
        if (r != hipSuccess) e = r;
    }
    return e;
}

}  // namespace pfbs
