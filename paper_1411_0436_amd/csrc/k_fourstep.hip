// Two-pass (four-step) spectrometer kernels for 4096 < N <= 2^20.
//
// N = N1 * N2, n = n1 + N1*n2, k = k2 + N2*k1:
//   X[k2 + N2 k1] = sum_n1 W_N1^(n1 k1) [ W_N^(n1 k2) sum_n2 y[n1 + N1 n2] W_N2^(n2 k2) ].
// Pass A (k_front_cols): unpack + pre-filter, the bracket for a tile of
//   T = 4096/N2 consecutive n1 (coalesced int8 rows), stored as
//   Z[j][pol][k2][n1].
// Pass B (k_back): for a tile of T = 4096/N1 consecutive k2, the outer sum
//   over n1 (contiguous rows of Z), the polarisation products and their
//   accumulation in registers over the spectra of a chunk; the chunk's sums
//   are written at u = k2*N1 + k1 (the reduction restores channel order).
#include "fft_common.h"

namespace pfbs {

template <int NPOL, bool PFB, int L>
__global__ __launch_bounds__(kTilePoints / 16 * NPOL) void k_front_cols(FrontArgs a) {
    typedef Geom<L> G;
    typedef typename Sample<NPOL>::word W;
    constexpr int NB = G::TPP * NPOL;
    constexpr int PTS = kTilePoints / NB;
    extern __shared__ float smem[];
    float *sre = smem;
    float *sim = smem + NPOL * G::plane;
    const int tid = threadIdx.x, pol = tid / G::TPP, lt = tid % G::TPP;
    // Workgroups are dealt to the 8 XCDs round-robin; give each XCD a
    // contiguous range of tiles and walk each tile's spectra consecutively, so
    // the workgroups that share an L2 share taps and frames.
    int tile, item;
    {
        const int nitems = gridDim.x / a.ntiles;
        if ((a.ntiles & 7) == 0) {
            const int xcd = blockIdx.x & 7, local = blockIdx.x >> 3;
            tile = xcd * (a.ntiles >> 3) + local / nitems;
            item = local % nitems;
        } else {
            tile = blockIdx.x % a.ntiles;
            item = blockIdx.x / a.ntiles;
        }
    }
    // spectra [js, je): the item-th run of ga spectra of the launch's range
    const long long js = a.sa0 + (long long)item * a.ga;
    const long long je = min(js + (long long)a.ga, a.sa1);
    const long long N = a.N;
    const int N1 = (int)a.N1;
    const int n1_0 = tile * G::T;
    const int P = PFB ? a.P : 1;
    const int c_own = lt >> (G::logL - 4), bb_own = lt & (G::L16 - 1);
    // W_N^(n1 k2) of this thread's column, k2 = bb + r*L/16
    const float2 *tw4 = a.tw4 + (unsigned)((n1_0 + c_own) * L + bb_own);

    for (long long j = js; j < je; ++j) {
        float2 y[PTS][NPOL];
#pragma unroll
        for (int s = 0; s < PTS; ++s)
#pragma unroll
            for (int pp = 0; pp < NPOL; ++pp) y[s][pp] = make_float2(0.f, 0.f);
        for (int p = 0; p < P; ++p) {
            // uniform bases, 32-bit unsigned per-lane offsets
            const W *fb = frame_ptr<NPOL>(a.fr, j + p, N) + n1_0;
            const float *hb = a.taps + (long long)p * N + n1_0;
#pragma unroll
            for (int s = 0; s < PTS; ++s) {
                const int i = tid + NB * s;
                const unsigned n = (unsigned)((i & (G::T - 1)) + N1 * (i >> G::logT));
                const W w = fb[n];
                if (PFB) tap_fma<NPOL>(y[s], hb[n], w);
                else Sample<NPOL>::unpack(w, y[s]);
            }
        }
#pragma unroll
        for (int s = 0; s < PTS; ++s) {
            const int i = tid + NB * s;
            const int c = i & (G::T - 1), n2 = i >> G::logT;
#pragma unroll
            for (int pp = 0; pp < NPOL; ++pp) {
                const int ad = G::idx(pp, c, n2);
                sre[ad] = y[s][pp].x;
                sim[ad] = y[s][pp].y;
            }
        }
        __syncthreads();
        float2 v[16];
        fft_plane<G>(sre, sim, pol, lt, a.g.tw, v);
        // ---- twiddle W_N^(n1 k2), back to LDS in natural order
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int k2 = bb_own + r * G::L16;
            const float2 z = cmul(v[r], tw4[r * G::L16]);
            const int ad = G::idx(pol, c_own, k2);
            sre[ad] = z.x;
            sim[ad] = z.y;
        }
        __syncthreads();
        // ---- coalesced store: T consecutive n1 of each (pol, k2) row
        float2 *zb = a.Z + (j - a.jz0) * NPOL * N + n1_0;
#pragma unroll
        for (int s = 0; s < (NPOL * kTilePoints) / NB; ++s) {
            const int i = tid + NB * s;
            const int cc = i & (G::T - 1);
            const int k2 = (i >> G::logT) & (L - 1);
            const int pp = i >> (G::logT + G::logL);
            const int ad = G::idx(pp, cc, k2);
            float2 *zp = zb + (unsigned)(pp * (int)N + k2 * N1 + cc);
            if (a.znt) {
                // streaming store: Z is read once, by the row pass
                float *zf = reinterpret_cast<float *>(zp);
                __builtin_nontemporal_store(sre[ad], zf);
                __builtin_nontemporal_store(sim[ad], zf + 1);
            } else {
                *zp = make_float2(sre[ad], sim[ad]);
            }
        }
        __syncthreads();
    }
}

// Row-pass tile: at least 1024 points per polarisation (64 threads each), so
// short rows still give many small workgroups.
template <int L> struct BackTile { static constexpr int TP = L < 1024 ? 1024 : L; };

template <int NPOL, int L>
__global__ __launch_bounds__(BackTile<L>::TP / 16 * NPOL) void k_back(BackArgs a) {
    typedef Geom<L, BackTile<L>::TP> G;
    constexpr int NB = G::TPP * NPOL;
    constexpr int NP = NPOL == 2 ? 4 : 1;
    constexpr int BINS = G::TP / NB;
    extern __shared__ float smem[];
    float *sre = smem;
    float *sim = smem + NPOL * G::plane;
    const int tid = threadIdx.x, pol = tid / G::TPP, lt = tid % G::TPP;
    const int tile = blockIdx.x % a.ntiles;
    const long long gid = a.ch.gid0 + blockIdx.x / a.ntiles;
    long long js, je;
    chunk_range(a.ch, gid, js, je);
    const long long N = a.N;
    const int k2_0 = tile * G::T;
    const int c_own = lt >> (G::logL - 4), bb_own = lt & (G::L16 - 1);

    float acc[BINS][NP];
#pragma unroll
    for (int i = 0; i < BINS; ++i)
#pragma unroll
        for (int q = 0; q < NP; ++q) acc[i][q] = 0.f;

    for (long long j = js; j < je; ++j) {
        const float2 *zb = a.Z + (j - a.jz0) * NPOL * N + (long long)k2_0 * L;
#pragma unroll
        for (int s = 0; s < (NPOL * G::TP) / NB; ++s) {
            const int i = tid + NB * s;
            const int n1 = i & (L - 1);
            const int cc = (i >> G::logL) & (G::T - 1);
            const int pp = i >> (G::logL + G::logT);
            const float2 *zp = zb + (unsigned)(pp * (int)N + cc * L + n1);
            const int ad = G::idx(pp, cc, n1);
            if (a.znt) {
                const float *zf = reinterpret_cast<const float *>(zp);
                sre[ad] = __builtin_nontemporal_load(zf);
                sim[ad] = __builtin_nontemporal_load(zf + 1);
            } else {
                const float2 z = *zp;
                sre[ad] = z.x;
                sim[ad] = z.y;
            }
        }
        __syncthreads();
        float2 v[16];
        fft_plane<G>(sre, sim, pol, lt, a.g.tw, v);
        if constexpr (NPOL == 2) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int ad = G::idx(pol, c_own, bb_own + r * G::L16);
                sre[ad] = v[r].x;
                sim[ad] = v[r].y;
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < BINS; ++i) {
                const int e = tid + NB * i;
                const int c = e >> G::logL, k = e & (L - 1);
                const int ax = G::idx(0, c, k), ay = G::idx(1, c, k);
                prod4(acc[i], make_float2(sre[ax], sim[ax]), make_float2(sre[ay], sim[ay]));
            }
            __syncthreads();
        } else {
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[r][0] += v[r].x * v[r].x + v[r].y * v[r].y;
        }
    }
    float *dst = a.part + (gid - a.ch.gid_lo) * (long long)NP * N;
    if constexpr (NPOL == 2) {
#pragma unroll
        for (int i = 0; i < BINS; ++i) {
            const int e = tid + NB * i;
            const int c = e >> G::logL, k1 = e & (L - 1);
            const long long u = (long long)(k2_0 + c) * L + k1;
#pragma unroll
            for (int q = 0; q < NP; ++q) dst[q * N + u] = acc[i][q];
        }
    } else {
        const long long u0 = (long long)(k2_0 + c_own) * L + bb_own;
#pragma unroll
        for (int r = 0; r < 16; ++r) dst[u0 + r * G::L16] = acc[r][0];
    }
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
