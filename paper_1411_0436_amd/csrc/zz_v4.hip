// Batched launches for several sub-bands: one launch per phase of a block.
// The paper's eight-sub-band mode runs its 16 FFTs in parallel (Section 4)
// and attributes small-N slowness to per-batch launch overhead (Section 5).
// Here a block of every sub-band is three launches: the front phase (single
// passes and column passes of all sub-bands), the row phase (all row passes)
// and the tail (dump reductions and tap histories, k_aux.hip).  Each
// workgroup finds its sub-band entry from its block id and runs the same
// device body as that sub-band's own kernel, so a batch gives the same bits
// as separate plans; the sub-bands' workgroups share the machine instead of
// queueing behind one another's partly filled launches.
#include "fft_bodies.h"

namespace pfbs {

template <class E>
__device__ __forceinline__ int find_entry(const E *t, int n, int bid) {
    int e = 0;
    while (e + 1 < n && bid >= t[e + 1].wg0) ++e;
    return e;
}

// LDS floats of one one-spectrum front workgroup (the host's front_lds_bytes).
template <int NPOL, int L>
constexpr int front_lds_floats() { return 2 * NPOL * (kTilePoints / L) * lds_pitch(L); }

// Single-pass entries of the front phase, in a function of their own: the
// single-pass bodies need more than the 128 registers a 1024-thread
// workgroup allows, and their spills stay inside this call instead of
// reaching the column-pass code of the kernel.
template <int NPOL>
__device__ __attribute__((noinline)) void front_single_entry(const FrontArgs &a, int vb, int tid, float *smem,
                                                             int half, int L, bool pfb) {
#define PFBS_BF_SINGLE(LL)                                                                                \
    if (L == LL) {                                                                                        \
        float *lds = smem + half * front_lds_floats<NPOL, LL>();                                          \
        if (pfb) front_single_body<NPOL, true, LL, 0, 0>(a, vb, tid, lds);                                \
        else front_single_body<NPOL, false, LL, 0, 0>(a, vb, tid, lds);                                   \
        return;                                                                                           \
    }
    PFBS_BF_SINGLE(16) PFBS_BF_SINGLE(32) PFBS_BF_SINGLE(64) PFBS_BF_SINGLE(128) PFBS_BF_SINGLE(256)
    PFBS_BF_SINGLE(512) PFBS_BF_SINGLE(1024) PFBS_BF_SINGLE(2048) PFBS_BF_SINGLE(4096)
#undef PFBS_BF_SINGLE
}

// Front phase.  A workgroup is twice the threads of a one-spectrum front
// kernel: a two-spectra column entry uses it whole, exactly as its own
// kernel; single-pass and one-spectrum column entries run two of their
// workgroups in it, one per half (whole waves), each half with its own LDS.
// Physical block b of an entry (entries start on multiples of 8, so b mod 8
// is the XCD) holds virtual blocks 16*(b/8) + 8*half + b mod 8: the XCD
// mapping of the column pass sees the same XCD as a plan's own launch, and
// the two halves of a CU take adjacent items (consecutive spectra of one
// column tile, which share frames in its cache).  The halves synchronise
// with workgroup barriers that both take part in; a half whose work ends
// first exits, and a barrier then waits only for the waves still running.
template <int NPOL>
__global__ __launch_bounds__(2 * kTilePoints / 16 * NPOL, 4) void k_batch_front(const BatchFrontEntry *__restrict__ t,
                                                                           int n) {
    extern __shared__ float smem[];
    if (n <= 0) return;
    const int e = find_entry(t, n, blockIdx.x);
    const int lb = blockIdx.x - t[e].wg0;
    if (lb < 0 || lb >= t[e].wgn) return;
    // a private copy: the body's global stores cannot alias it
    FrontArgs a = t[e].a;
    globalise(a);
    const int kind = t[e].kind, L = t[e].L, pt = t[e].pt, items = t[e].items;
    const bool pfb = t[e].pfb != 0;
    if (kind == 2) {
#define PFBS_BF_PAIR(LL)                                                                                  \
    if (L == LL) {                                                                                        \
        if (pt == 4) front_cols_pair_body<NPOL, LL, 4, 0>(a, lb, items, threadIdx.x, smem);               \
        else if (pt == 8) front_cols_pair_body<NPOL, LL, 8, 0>(a, lb, items, threadIdx.x, smem);          \
        else front_cols_pair_body<NPOL, LL, 0, 0>(a, lb, items, threadIdx.x, smem);                       \
        return;                                                                                           \
    }
        PFBS_BF_PAIR(64) PFBS_BF_PAIR(128) PFBS_BF_PAIR(256)
#undef PFBS_BF_PAIR
        return;
    }
    constexpr int HALF = kTilePoints / 16 * NPOL;
    // wave-uniform: whole waves make up each half
    const int half = __builtin_amdgcn_readfirstlane((int)threadIdx.x) >= HALF ? 1 : 0;
    const int vb = ((lb >> 3) << 4) + (half << 3) + (lb & 7);
    if (vb >= items) return;
    const int tid = (int)threadIdx.x - half * HALF;
    if (kind == 0) {
        front_single_entry<NPOL>(a, vb, tid, smem, half, L, pfb);
        return;
    }
#define PFBS_BF_COLS(LL)                                                                                  \
    if (L == LL) {                                                                                        \
        float *lds = smem + half * front_lds_floats<NPOL, LL>();                                          \
        if (!pfb) front_cols_body<NPOL, false, LL, 0, 0>(a, vb, items, tid, lds);                         \
        else if (pt == 4) front_cols_body<NPOL, true, LL, 0, 4>(a, vb, items, tid, lds);                  \
        else if (pt == 8) front_cols_body<NPOL, true, LL, 0, 8>(a, vb, items, tid, lds);                  \
        else front_cols_body<NPOL, true, LL, 0, 0>(a, vb, items, tid, lds);                               \
        return;                                                                                           \
    }
    PFBS_BF_COLS(64) PFBS_BF_COLS(128) PFBS_BF_COLS(256) PFBS_BF_COLS(512)
#undef PFBS_BF_COLS
}

// Row phase: every row length and row arithmetic of a batch at one tile of
// TP points per polarisation (TP / L rows per workgroup step).
template <int NPOL, int TP>
__global__ __launch_bounds__(TP / 16 * NPOL) void k_batch_back(const BatchBackEntry *__restrict__ t, int n) {
    extern __shared__ float smem[];
    if (n <= 0) return;
    const int e = find_entry(t, n, blockIdx.x);
    const int lb = blockIdx.x - t[e].wg0;
    if (lb < 0 || lb >= t[e].wgn) return;
    BackArgs a = t[e].a;
    globalise(a);
    const int L = t[e].L, prec = t[e].prec;
#define PFBS_BB(LL)                                                                                       \
    if constexpr (LL <= TP) {                                                                             \
        if (L == LL) {                                                                                    \
            if (prec == 3) back_body<NPOL, LL, 3, TP>(a, lb, threadIdx.x, smem);                          \
            else if (prec == 2) back_body<NPOL, LL, 2, TP>(a, lb, threadIdx.x, smem);                     \
            else back_body<NPOL, LL, 0, TP>(a, lb, threadIdx.x, smem);                                    \
            return;                                                                                       \
        }                                                                                                 \
    }
    PFBS_BB(32) PFBS_BB(64) PFBS_BB(128) PFBS_BB(256) PFBS_BB(512) PFBS_BB(1024) PFBS_BB(2048) PFBS_BB(4096)
#undef PFBS_BB
}

const void *batch_front_fn(int npol) {
    return npol == 2 ? reinterpret_cast<const void *>(&k_batch_front<2>)
                     : reinterpret_cast<const void *>(&k_batch_front<1>);
}

const void *batch_back_fn(int npol, int tp) {
    switch (tp) {
    case 1024: return npol == 2 ? reinterpret_cast<const void *>(&k_batch_back<2, 1024>)
                                : reinterpret_cast<const void *>(&k_batch_back<1, 1024>);
    case 2048: return npol == 2 ? reinterpret_cast<const void *>(&k_batch_back<2, 2048>)
                                : reinterpret_cast<const void *>(&k_batch_back<1, 2048>);
    case 4096: return npol == 2 ? reinterpret_cast<const void *>(&k_batch_back<2, 4096>)
                                : reinterpret_cast<const void *>(&k_batch_back<1, 4096>);
    default: return nullptr;
    }
}

bool init_batch(int lds_limit) {
    bool ok = true;
    for (int npol = 1; npol <= 2; ++npol) {
        if (hipFuncSetAttribute(batch_front_fn(npol), hipFuncAttributeMaxDynamicSharedMemorySize, lds_limit) !=
            hipSuccess)
            ok = false;
        for (int tp : {1024, 2048, 4096})
            if (hipFuncSetAttribute(batch_back_fn(npol, tp), hipFuncAttributeMaxDynamicSharedMemorySize, lds_limit) !=
                hipSuccess)
                ok = false;
    }
    return ok;
}

}  // namespace pfbs
