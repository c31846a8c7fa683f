// Single-pass spectrometer kernel for N <= 4096: unpack + polyphase
// pre-filter + the whole N-point FFT + polarisation products + accumulation,
// one kernel per block (paper, Section 4: pre-filtering, parallel FFTs and
// accumulation of the per-block loop).
//
// A workgroup owns one chunk of consecutive spectra.  Each step takes
// T = 4096/N consecutive spectra as the T columns of the batched LDS FFT; a
// thread accumulates the products of fixed output bins of one column in
// registers; at the end of the chunk the T columns are summed in column order
// and written as the chunk's partial sum.
#include "fft_common.h"

namespace pfbs {

template <int NPOL, bool PFB, int L>
__global__ __launch_bounds__(kTilePoints / 16 * NPOL) void k_front_single(FrontArgs a) {
    typedef Geom<L> G;
    typedef typename Sample<NPOL>::word W;
    constexpr int NB = G::TPP * NPOL;      // threads
    constexpr int PTS = kTilePoints / NB;  // pre-filter points per thread (all pols each)
    constexpr int NP = NPOL == 2 ? 4 : 1;  // products
    constexpr int BINS = kTilePoints / NB; // accumulated bins per thread
    extern __shared__ float smem[];
    float *sre = smem;
    float *sim = smem + NPOL * G::plane;
    const int tid = threadIdx.x, pol = tid / G::TPP, lt = tid % G::TPP;
    const long long gid = a.ch.gid0 + blockIdx.x;
    long long js, je;
    chunk_range(a.ch, gid, js, je);
    const int P = PFB ? a.P : 1;
    // column and butterfly owned in the last radix-16 pass
    const int c_own = lt >> (G::logL - 4), bb_own = lt & (G::L16 - 1);

    float acc[BINS][NP];
#pragma unroll
    for (int i = 0; i < BINS; ++i)
#pragma unroll
        for (int q = 0; q < NP; ++q) acc[i][q] = 0.f;

    for (long long j0 = js; j0 < je; j0 += G::T) {
        // ---- unpack + pre-filter (points along n: coalesced) into LDS
        float2 y[PTS][NPOL];
#pragma unroll
        for (int s = 0; s < PTS; ++s)
#pragma unroll
            for (int pp = 0; pp < NPOL; ++pp) y[s][pp] = make_float2(0.f, 0.f);
        for (int p = 0; p < P; ++p) {
#pragma unroll
            for (int s = 0; s < PTS; ++s) {
                const int i = tid + NB * s;
                const int c = i >> G::logL, n = i & (L - 1);
                const long long jj = j0 + c;
                if (jj < je) {
                    const W w = frame_ptr<NPOL>(a.fr, jj + p, L)[n];
                    if (PFB) {
                        tap_fma<NPOL>(y[s], a.taps[p * L + n], w);
                    } else {
                        Sample<NPOL>::unpack(w, y[s]);
                    }
                }
            }
        }
#pragma unroll
        for (int s = 0; s < PTS; ++s) {
            const int i = tid + NB * s;
            const int c = i >> G::logL, n = i & (L - 1);
#pragma unroll
            for (int pp = 0; pp < NPOL; ++pp) {
                const int ad = G::idx(pp, c, n);
                sre[ad] = y[s][pp].x;
                sim[ad] = y[s][pp].y;
            }
        }
        __syncthreads();
        float2 v[16];
        fft_plane<G>(sre, sim, pol, lt, a.g.tw, v);
        if constexpr (NPOL == 2) {
            // X and Y of a bin meet through LDS (natural order)
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
                if (j0 + c < je) {
                    const int ax = G::idx(0, c, k), ay = G::idx(1, c, k);
                    prod4(acc[i], make_float2(sre[ax], sim[ax]), make_float2(sre[ay], sim[ay]));
                }
            }
            __syncthreads();
        } else {
            if (j0 + c_own < je) {
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[r][0] += v[r].x * v[r].x + v[r].y * v[r].y;
            }
        }
    }
    // ---- sum the T columns in column order; write the chunk's partial
    __syncthreads();
    float *red = smem;  // [T][NP][L]
    if constexpr (NPOL == 2) {
#pragma unroll
        for (int i = 0; i < BINS; ++i) {
            const int e = tid + NB * i;
            const int c = e >> G::logL, k = e & (L - 1);
#pragma unroll
            for (int q = 0; q < NP; ++q) red[(c * NP + q) * L + k] = acc[i][q];
        }
    } else {
#pragma unroll
        for (int r = 0; r < 16; ++r) red[c_own * L + bb_own + r * G::L16] = acc[r][0];
    }
    __syncthreads();
    float *dst = a.part + (gid - a.ch.gid_lo) * (long long)NP * L;
    for (int e = tid; e < NP * L; e += NB) {
        float s = 0.f;
#pragma unroll 4
        for (int c = 0; c < G::T; ++c) s += red[c * NP * L + e];
        dst[e] = s;
    }
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
