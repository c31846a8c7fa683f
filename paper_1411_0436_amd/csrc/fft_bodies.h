// Kernel bodies as device functions of a virtual block id, so that the same
// code serves a plan's own launches and the batched multi-sub-band launches.
#pragma once

#include "fft_common.h"

namespace pfbs {

// Single-pass spectrometer body for N <= 4096: unpack + polyphase
// pre-filter + the whole N-point FFT + polarisation products + accumulation
// (paper, Section 4: pre-filtering, parallel FFTs and accumulation of the
// per-block loop).  A workgroup owns one chunk of consecutive spectra.  Each
// step takes T = 4096/N consecutive spectra as the T columns of the batched
// LDS FFT; a thread accumulates the products of fixed output bins of one
// column in registers; at the end of the chunk the T columns are summed in
// column order and written as the chunk's partial sum.
template <int NPOL, bool PFB, int L, int PREC = 0, int PT = 0>
__device__ __forceinline__ void front_single_body(const FrontArgs &a, int bid, int tid, float *smem) {
    typedef Geom<L, kTilePoints, 5> G;
    typedef typename Sample<NPOL>::word4 W4;
    constexpr int NB = G::TPP * NPOL;      // threads
    constexpr int PTS = kTilePoints / NB;  // pre-filter points per thread (all pols each)
    constexpr int NP = NPOL == 2 ? 4 : 1;  // products
    constexpr int BINS = kTilePoints / NB; // accumulated bins per thread
    float *sre = smem;
    float *sim = smem + NPOL * G::plane;
    const int pol = tid / G::TPP, lt = tid % G::TPP;
    const long long gid = a.ch.gid0 + bid;
    long long js, je;
    chunk_range(a.ch, gid, js, je);
    const int P = PFB ? a.P : 1;
    // column and butterfly owned in the last radix-16 pass
    const int c_own = lt >> (G::logL - 4), bb_own = lt & (G::L16 - 1);
    MfmaW Wm{};
    if constexpr (PREC != 0) Wm = mfma_operands_load(a.g.mw, lt & 63);

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
        // work item q: four consecutive points 4q .. 4q+3 of the T columns
        if constexpr (PFB && PT > 0) {
            // compile-time tap count: the loads of tap p+1 go out before the
            // multiply-adds of tap p, in registers of their own.  Columns past
            // the chunk read the frames of its last spectrum (valid memory);
            // their outputs are never accumulated.
            typedef typename Sample<NPOL>::word W;
            auto loads = [&](int p, W4 (&w4)[PTS / 4], float4 (&h4)[PTS / 4]) {
#pragma unroll
                for (int g = 0; g < PTS / 4; ++g) {
                    const int i = 4 * (tid + NB * g);
                    const int c = i >> G::logL, n = i & (L - 1);
                    const long long jj = min(j0 + c, je - 1);
                    const W *fb = frame_ptr<NPOL>(a.fr, jj + p, L);
                    w4[g] = *reinterpret_cast<const W4 *>(fb + n);
                    h4[g] = *reinterpret_cast<const float4 *>(a.taps + p * L + n);
                }
            };
            W4 wq[PT][PTS / 4];
            float4 hq[PT][PTS / 4];
            loads(0, wq[0], hq[0]);
#pragma unroll
            for (int p = 0; p < PT; ++p) {
                if (p + 1 < PT) loads(p + 1, wq[p + 1], hq[p + 1]);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int g = 0; g < PTS / 4; ++g)
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        tap_fma<NPOL>(y[4 * g + e], part4(hq[p][g], e), Sample<NPOL>::part(wq[p][g], e));
            }
        } else {
            for (int p = 0; p < P; ++p) {
#pragma unroll
                for (int g = 0; g < PTS / 4; ++g) {
                    const int i = 4 * (tid + NB * g);
                    const int c = i >> G::logL, n = i & (L - 1);
                    const long long jj = j0 + c;
                    if (jj < je) {
                        const W4 w4 = *reinterpret_cast<const W4 *>(frame_ptr<NPOL>(a.fr, jj + p, L) + n);
                        if (PFB) {
                            const float4 h4 = *reinterpret_cast<const float4 *>(a.taps + p * L + n);
#pragma unroll
                            for (int e = 0; e < 4; ++e)
                                tap_fma<NPOL>(y[4 * g + e], part4(h4, e), Sample<NPOL>::part(w4, e));
                        } else {
#pragma unroll
                            for (int e = 0; e < 4; ++e) Sample<NPOL>::unpack(Sample<NPOL>::part(w4, e), y[4 * g + e]);
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int g = 0; g < PTS / 4; ++g) {
            const int i = 4 * (tid + NB * g);
            const int c = i >> G::logL, n = i & (L - 1);
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int pp = 0; pp < NPOL; ++pp) {
                    const int ad = G::idx(pp, c, n + e);
                    sre[ad] = y[4 * g + e][pp].x;
                    sim[ad] = y[4 * g + e][pp].y;
                }
        }
        __syncthreads();
        float2 v[16];
        fft_plane_p<G, PREC>(sre, sim, pol, lt, a.g.tw, Wm, v, NPOL == 1);
        if constexpr (NPOL == 2) {
            // X and Y of a bin meet through LDS (natural order)
            if constexpr (!FftPrec<PREC>::IN_LDS) {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int ad = G::idx(pol, c_own, bb_own + r * G::L16);
                    sre[ad] = v[r].x;
                    sim[ad] = v[r].y;
                }
                __syncthreads();
            }
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
            // v was read back from LDS, which the next step overwrites
            if constexpr (FftPrec<PREC>::IN_LDS || FftWave<G, PREC>::value) __syncthreads();
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

// Two-pass (four-step) bodies for 4096 < N <= 2^20.
//
// N = N1 * N2, n = n1 + N1*n2, k = k2 + N2*k1:
//   X[k2 + N2 k1] = sum_n1 W_N1^(n1 k1) [ W_N^(n1 k2) sum_n2 y[n1 + N1 n2] W_N2^(n2 k2) ].
// Column pass: unpack + pre-filter, the bracket for a tile of T = 4096/N2
//   consecutive n1 (coalesced int8 rows), stored as Z[j][pol][k2][n1].
// Row pass: for a tile of consecutive k2, the outer sum over n1 (contiguous
//   rows of Z), the polarisation products and their accumulation in registers
//   over the spectra of a chunk; the chunk's sums are written at
//   u = k2*N1 + k1 (the reduction restores channel order).
// Column-pass workgroup -> (column tile, run of spectra).  Workgroups are
// dealt to the 8 XCDs round-robin; give each XCD a contiguous range of tiles
// and walk each tile's spectra consecutively, so the workgroups that share an
// L2 share taps and frames.  Tiles whose int8 row segments are narrower than
// a 128-byte line run as a group of TGW adjacent tiles that together fill the
// line, spectrum by spectrum.  With fewer than 8 such groups, each group's
// spectra are split between 8/groups XCDs instead (a line never straddles two
// L2s; only the P-1 frames at a split are fetched twice).  Needs the item
// count to be a multiple of 8, which the plan pads (padded items are empty).
template <int T, int NPOL>
__device__ __forceinline__ void cols_tile_item(int ntiles, int bid, int nblk, int &tile, int &item) {
    const int nitems = nblk / ntiles;
    constexpr int SEG = T * 2 * NPOL;  // bytes of a tile's row segment
    constexpr int TGW = SEG >= 128 ? 1 : 128 / SEG;
    const int xcd = bid & 7, local = bid >> 3;
    const int ngroups = ntiles / TGW;
    if ((ntiles & 7) == 0 && (ntiles >> 3) % TGW == 0) {
        const int tpx = ntiles >> 3;
        const int grp = local / (TGW * nitems), rem = local - grp * (TGW * nitems);
        tile = xcd * tpx + grp * TGW + rem % TGW;
        item = rem / TGW;
    } else if (ngroups > 0 && ntiles % TGW == 0 && 8 % ngroups == 0 && nitems % (8 / ngroups) == 0) {
        const int per = nitems / (8 / ngroups);
        tile = (xcd % ngroups) * TGW + local % TGW;
        item = (xcd / ngroups) * per + local / TGW;
    } else if ((ntiles & 7) == 0) {
        const int tpx = ntiles >> 3;
        int TG = TGW;
        while (tpx % TG) TG >>= 1;
        const int grp = local / (TG * nitems), rem = local - grp * (TG * nitems);
        tile = xcd * tpx + grp * TG + rem % TG;
        item = rem / TG;
    } else {
        tile = bid % ntiles;
        item = bid / ntiles;
    }
}

template <int NPOL, bool PFB, int L, int PREC = 0, int PT = 0>
__device__ __forceinline__ void front_cols_body(const FrontArgs &a, int bid, int nblk, int tid, float *smem) {
    typedef Geom<L> G;
    typedef typename Sample<NPOL>::word W;
    constexpr int NB = G::TPP * NPOL;
    constexpr int PTS = G::TP / NB;
    float *sre = smem;
    float *sim = smem + NPOL * G::plane;
    const int pol = tid / G::TPP, lt = tid % G::TPP;
    int tile, item;
    cols_tile_item<G::T, NPOL>(a.ntiles, bid, nblk, tile, item);
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
    MfmaW Wm{};
    if constexpr (PREC != 0) Wm = mfma_operands_load(a.g.mw, lt & 63);

    // pre-filter work item q: four consecutive columns 4*(q mod T/4) .. +3 of
    // row n2 = q / (T/4), read with one 16-byte access per frame and per tap row
    static_assert(G::T % 4 == 0 && PTS % 4 == 0, "column tile of whole 4-sample groups");
    typedef typename Sample<NPOL>::word4 W4;
    for (long long j = js; j < je; ++j) {
        float2 y[PTS][NPOL];
#pragma unroll
        for (int s = 0; s < PTS; ++s)
#pragma unroll
            for (int pp = 0; pp < NPOL; ++pp) y[s][pp] = make_float2(0.f, 0.f);
        // uniform bases, 32-bit unsigned per-lane offsets
        // uniform bases, 32-bit unsigned per-lane offsets (global loads
        // measured faster here than buffer loads: C2 column pass 131 against
        // 137 us, split-FP16 at N=2^19 761 against 908 us)
        auto tap_loads = [&](int p, W4 (&w4)[PTS / 4], float4 (&h4)[PTS / 4]) {
            const W *fb = frame_ptr<NPOL>(a.fr, j + p, N) + n1_0;
            const float *hb = a.taps + (long long)p * N + n1_0;
#pragma unroll
            for (int g = 0; g < PTS / 4; ++g) {
                const int q = tid + NB * g;
                const unsigned n = (unsigned)(4 * (q & (G::T / 4 - 1)) + N1 * (q >> (G::logT - 2)));
                w4[g] = *reinterpret_cast<const W4 *>(fb + n);
                if (PFB) h4[g] = *reinterpret_cast<const float4 *>(hb + n);
            }
        };
        W4 w4[PTS / 4];
        float4 h4[PTS / 4];
        tap_loads(0, w4, h4);
        if constexpr (!PFB) {
#pragma unroll
            for (int g = 0; g < PTS / 4; ++g)
#pragma unroll
                for (int e = 0; e < 4; ++e) Sample<NPOL>::unpack(Sample<NPOL>::part(w4[g], e), y[4 * g + e]);
        } else if constexpr (PT > 0) {
            // compile-time tap count, fully unrolled: tap p+1's loads go out
            // before tap p's multiply-adds, each tap in registers of its own,
            // and the scheduler may not move them across (a rolled loop made
            // the compiler wait for the next tap's loads at the end of every
            // iteration, to copy them into the loop-carried registers)
            W4 wq[PT][PTS / 4];
            float4 hq[PT][PTS / 4];
#pragma unroll
            for (int g = 0; g < PTS / 4; ++g) {
                wq[0][g] = w4[g];
                hq[0][g] = h4[g];
            }
#pragma unroll
            for (int p = 0; p < PT; ++p) {
                if (p + 1 < PT) tap_loads(p + 1, wq[p + 1], hq[p + 1]);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int g = 0; g < PTS / 4; ++g)
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        tap_fma<NPOL>(y[4 * g + e], part4(hq[p][g], e), Sample<NPOL>::part(wq[p][g], e));
            }
        } else {
            for (int p = 0; p < P; ++p) {
                // the next tap's loads go out before this tap's arithmetic, so
                // one tap's memory latency overlaps the previous tap's FMAs
                // (the last tap reloads itself, from cache, to keep the loop
                // branch-free)
                W4 w4n[PTS / 4];
                float4 h4n[PTS / 4];
                tap_loads(min(p + 1, P - 1), w4n, h4n);
#pragma unroll
                for (int g = 0; g < PTS / 4; ++g) {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        tap_fma<NPOL>(y[4 * g + e], part4(h4[g], e), Sample<NPOL>::part(w4[g], e));
                    w4[g] = w4n[g];
                    h4[g] = h4n[g];
                }
            }
        }
#pragma unroll
        for (int g = 0; g < PTS / 4; ++g) {
            const int q = tid + NB * g;
            const int c0 = 4 * (q & (G::T / 4 - 1)), n2 = q >> (G::logT - 2);
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int pp = 0; pp < NPOL; ++pp) {
                    const int ad = G::idx(pp, c0 + e, n2);
                    sre[ad] = y[4 * g + e][pp].x;
                    sim[ad] = y[4 * g + e][pp].y;
                }
        }
        __syncthreads();
        float2 v[16];
        fft_plane_p<G, PREC, true>(sre, sim, pol, lt, a.g.tw, Wm, v, true);
        // ---- twiddle W_N^(n1 k2), back to LDS in natural order (each thread
        // rewrites the positions it has just read)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int k2 = bb_own + r * G::L16;
            const float2 z = cmul(v[r], tw4[r * G::L16]);
            const int ad = G::idx(pol, c_own, k2);
            sre[ad] = z.x;
            sim[ad] = z.y;
        }
        __syncthreads();
        // ---- coalesced store: T consecutive n1 of each (pol, k2) row, two
        // complex values (16 bytes) per access
        float2 *zb = a.Z + (j - a.jz0) * NPOL * N + n1_0;
#pragma unroll
        for (int s = 0; s < (NPOL * G::TP) / (2 * NB); ++s) {
            const int i = tid + NB * s;
            const int cc = 2 * (i & (G::T / 2 - 1));
            const int k2 = (i >> (G::logT - 1)) & (L - 1);
            const int pp = i >> (G::logT - 1 + G::logL);
            const int ad0 = G::idx(pp, cc, k2), ad1 = G::idx(pp, cc + 1, k2);
            const floatx4 v = {sre[ad0], sim[ad0], sre[ad1], sim[ad1]};
            floatx4 *zp = reinterpret_cast<floatx4 *>(zb + (unsigned)(pp * (int)N + k2 * N1 + cc));
            if (a.znt) __builtin_nontemporal_store(v, zp);  // Z is read once, by the row pass
            else *zp = v;
        }
        __syncthreads();
    }
}

// Column pass with pre-filter, two consecutive spectra j and j+1 per
// workgroup step (twice the threads and LDS of front_cols_body), the FFT in
// any precision of front_cols_body.  The
// pre-filter reads most of its bytes from L2 (P frames and P tap rows per
// point), so each thread filters its points for both spectra at once: one
// load of tap row p serves both, and the frames slide (frame j+p+1 is the
// second spectrum's tap p and the first's tap p+1), P+2 frame loads for two
// spectra instead of 2P.  Each half of the workgroup then transforms and
// stores one spectrum, exactly as front_cols_body does (same arithmetic in
// the same order, so the same bits).
template <int NPOL, int L, int PT = 0, int PREC = 0>
__device__ __forceinline__ void front_cols_pair_body(const FrontArgs &a, int bid, int nblk, int tid, float *smem) {
    typedef Geom<L> G;
    typedef typename Sample<NPOL>::word W;
    typedef typename Sample<NPOL>::word4 W4;
    constexpr int NB = G::TPP * NPOL;   // threads per spectrum
    constexpr int GRP = G::TP / (8 * NB);  // 4-point groups per thread and spectrum
    static_assert(G::T % 4 == 0 && GRP >= 1 && GRP * 8 * NB == G::TP, "pair tile of whole 4-sample groups");
    const int half = tid / NB, t = tid - half * NB;
    const int pol = t / G::TPP, lt = t % G::TPP;
    float *sre = smem + half * (2 * NPOL * G::plane);
    float *sim = sre + NPOL * G::plane;
    int tile, item;
    cols_tile_item<G::T, NPOL>(a.ntiles, bid, nblk, tile, item);
    // spectra [js, je): the item-th run of 2*ga spectra of the launch's range
    const long long js = a.sa0 + (long long)item * 2 * a.ga;
    const long long je = min(js + 2LL * a.ga, a.sa1);
    const long long N = a.N;
    const int N1 = (int)a.N1;
    const int n1_0 = tile * G::T;
    const int P = a.P;
    const int c_own = lt >> (G::logL - 4), bb_own = lt & (G::L16 - 1);
    const float2 *tw4 = a.tw4 + (unsigned)((n1_0 + c_own) * L + bb_own);
    MfmaW Wm{};
    if constexpr (PREC != 0) Wm = mfma_operands_load(a.g.mw, lt & 63);

    for (long long j = js; j < je; j += 2) {
        const bool two = j + 1 < je;
        // last frame read by a spectrum of this step (reads past it are
        // clamped to it and their results unused)
        const long long f_last = j + (two ? 1 : 0) + P - 1;
        float2 y[2][4 * GRP][NPOL];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int s = 0; s < 4 * GRP; ++s)
#pragma unroll
                for (int pp = 0; pp < NPOL; ++pp) y[h][s][pp] = make_float2(0.f, 0.f);
        // buffer loads: uniform frame / tap-row base in a scalar descriptor,
        // 32-bit per-lane offsets (no 64-bit address per load held in vector
        // registers; N=2^19 column pass 658 -> 522 us against global loads)
        const unsigned rest = (unsigned)(N - n1_0);   // points from the tile's first column to the frame end
        auto frame_loads = [&](long long f, W4 (&w4)[GRP]) {
            const Rsrc fr = make_rsrc(frame_ptr<NPOL>(a.fr, min(f, f_last), N) + n1_0, rest * (unsigned)sizeof(W));
#pragma unroll
            for (int g = 0; g < GRP; ++g) {
                const int q = tid + 2 * NB * g;
                const unsigned n = (unsigned)(4 * (q & (G::T / 4 - 1)) + N1 * (q >> (G::logT - 2)));
                w4[g] = buf_load<W4>(fr, n * (unsigned)sizeof(W));
            }
        };
        auto tap_loads = [&](int p, float4 (&h4)[GRP]) {
            const Rsrc hr = make_rsrc(a.taps + (long long)p * N + n1_0, rest * 4u);
#pragma unroll
            for (int g = 0; g < GRP; ++g) {
                const int q = tid + 2 * NB * g;
                const unsigned n = (unsigned)(4 * (q & (G::T / 4 - 1)) + N1 * (q >> (G::logT - 2)));
                h4[g] = buf_load<float4>(hr, n * 4u);
            }
        };
        // xa: frame j+p (first spectrum's tap p), xb: frame j+p+1 (second's)
        if constexpr (PT > 0) {
            // compile-time tap count, fully unrolled: frame j+p+2 and tap p+1
            // are loaded before step p's multiply-adds, in registers of their own
            W4 xf[PT + 1][GRP];
            float4 hq[PT][GRP];
            frame_loads(j, xf[0]);
            frame_loads(j + 1, xf[1]);
            tap_loads(0, hq[0]);
#pragma unroll
            for (int p = 0; p < PT; ++p) {
                if (p + 2 <= PT) frame_loads(j + p + 2, xf[p + 2]);
                if (p + 1 < PT) tap_loads(p + 1, hq[p + 1]);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int g = 0; g < GRP; ++g)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        tap_fma<NPOL>(y[0][4 * g + e], part4(hq[p][g], e), Sample<NPOL>::part(xf[p][g], e));
                        tap_fma<NPOL>(y[1][4 * g + e], part4(hq[p][g], e), Sample<NPOL>::part(xf[p + 1][g], e));
                    }
            }
        } else {
        W4 xa[GRP], xb[GRP];
        float4 h4[GRP];
        frame_loads(j, xa);
        frame_loads(j + 1, xb);
        tap_loads(0, h4);
        for (int p = 0; p < P; ++p) {
            // next step's loads before this step's arithmetic
            W4 xn[GRP];
            float4 hn[GRP];
            frame_loads(j + p + 2, xn);
            tap_loads(min(p + 1, P - 1), hn);
#pragma unroll
            for (int g = 0; g < GRP; ++g) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    tap_fma<NPOL>(y[0][4 * g + e], part4(h4[g], e), Sample<NPOL>::part(xa[g], e));
                    tap_fma<NPOL>(y[1][4 * g + e], part4(h4[g], e), Sample<NPOL>::part(xb[g], e));
                }
                xa[g] = xb[g];
                xb[g] = xn[g];
                h4[g] = hn[g];
            }
        }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            float *hre = smem + h * (2 * NPOL * G::plane), *him = hre + NPOL * G::plane;
#pragma unroll
            for (int g = 0; g < GRP; ++g) {
                const int q = tid + 2 * NB * g;
                const int c0 = 4 * (q & (G::T / 4 - 1)), n2 = q >> (G::logT - 2);
#pragma unroll
                for (int e = 0; e < 4; ++e)
#pragma unroll
                    for (int pp = 0; pp < NPOL; ++pp) {
                        const int ad = G::idx(pp, c0 + e, n2);
                        hre[ad] = y[h][4 * g + e][pp].x;
                        him[ad] = y[h][4 * g + e][pp].y;
                    }
            }
        }
        __syncthreads();
        float2 v[16];
        fft_plane_p<G, PREC, true>(sre, sim, pol, lt, a.g.tw, Wm, v, true);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int k2 = bb_own + r * G::L16;
            const float2 z = cmul(v[r], tw4[r * G::L16]);
            const int ad = G::idx(pol, c_own, k2);
            sre[ad] = z.x;
            sim[ad] = z.y;
        }
        __syncthreads();
        if (half == 0 || two) {
            float2 *zb = a.Z + (j + half - a.jz0) * NPOL * N + n1_0;
#pragma unroll
            for (int s = 0; s < (NPOL * G::TP) / (2 * NB); ++s) {
                const int i = t + NB * s;
                const int cc = 2 * (i & (G::T / 2 - 1));
                const int k2 = (i >> (G::logT - 1)) & (L - 1);
                const int pp = i >> (G::logT - 1 + G::logL);
                const int ad0 = G::idx(pp, cc, k2), ad1 = G::idx(pp, cc + 1, k2);
                const floatx4 v = {sre[ad0], sim[ad0], sre[ad1], sim[ad1]};
                floatx4 *zp = reinterpret_cast<floatx4 *>(zb + (unsigned)(pp * (int)N + k2 * N1 + cc));
                if (a.znt) __builtin_nontemporal_store(v, zp);
                else *zp = v;
            }
        }
        __syncthreads();
    }
}

// Row-pass tile: at least 1024 points per polarisation (64 threads each), so
// short rows still give many small workgroups.
template <int L> struct BackTile { static constexpr int TP = back_tile_points(L); };
// LDS padding of the row pass (Geom): PS = 5 measured faster except for FP32
// rows of 512 points and more (N = 2^17: row pass 0.113 -> 0.093 ms with PS = 4).
template <int L, int PREC> struct BackPad {
    static constexpr int PS = ((PREC == 0 || PREC == 3) && L >= 512) ? 4 : 5;
};

// The row kernels loop over the spectra of a chunk with the same lane
// indices in every iteration, and the compiler hoists every LDS offset derived
// from them out of the loop, holding them in registers for the whole kernel.
// For the matrix-core and FP64 rows the lane index is passed through an empty
// asm statement at each iteration, so the offsets are recomputed per spectrum
// instead (the split-FP16 kernel on 2048-point rows: 224 -> 125 VGPRs, two ->
// four waves per SIMD, row pass -5 %); the FP32 rows, whose registers go to
// the next spectrum's prefetched intermediate, measured faster with them
// hoisted.
template <int PREC> struct FreshIdx { static constexpr bool value = PREC != 0; };
__device__ __forceinline__ int opaque_int(int x) {
    asm volatile("" : "+v"(x));
    return x;
}

// PREC 3: the row FFT and the products in FP64 on the vector ALUs (each
// product rounded once to FP32 before it is accumulated); the intermediate
// stays FP32.  A strong tone's energy sits in one intermediate row, and an
// FP32 row FFT spreads its rounding over every channel of that row.
// TP: row-pass tile points (the plan's own launches use BackTile<L>::TP; a
// batched launch runs every row length of a batch at one tile size, which
// changes only how rows are grouped into workgroups, not their arithmetic).
template <int NPOL, int L, int PREC = 0, int TP = BackTile<L>::TP>
__device__ __forceinline__ void back_body(const BackArgs &a, int bid, int tid, float *smem) {
    typedef Geom<L, TP, BackPad<L, PREC>::PS> G;
    constexpr bool F64 = PREC == 3;
    typedef std::conditional_t<F64, double, float> T;
    typedef typename Cplx<T>::type C;
    constexpr int NB = G::TPP * NPOL;
    constexpr int NP = NPOL == 2 ? 4 : 1;
    constexpr int BINS = G::TP / NB;
    T *sre = reinterpret_cast<T *>(smem);
    T *sim = sre + NPOL * G::plane;
    const int pol = tid / G::TPP, lt = tid % G::TPP;
    const int tile = bid % a.ntiles;
    const long long gid = a.ch.gid0 + bid / a.ntiles;
    long long js, je;
    chunk_range(a.ch, gid, js, je);
    const long long N = a.N;
    const int k2_0 = tile * G::T;
    const int c_own = lt >> (G::logL - 4), bb_own = lt & (G::L16 - 1);
    MfmaW Wm{};
    if constexpr (FftPrec<PREC>::IN_LDS) Wm = mfma_operands_load(a.g.mw, lt & 63);

    float acc[BINS][NP];
#pragma unroll
    for (int i = 0; i < BINS; ++i)
#pragma unroll
        for (int q = 0; q < NP; ++q) acc[i][q] = 0.f;

    // FP32 rows: the next spectrum's intermediate is loaded into registers
    // while this one is transformed (two consecutive n1, 16 bytes, per access)
    constexpr bool ZPRE = PREC == 0;
    constexpr int NZ = (NPOL * G::TP) / (2 * NB);
    auto z_loads = [&](long long jj, floatx4 (&z)[NZ]) {
        const float2 *zb = a.Z + (jj - a.jz0) * NPOL * N + (long long)k2_0 * L;
#pragma unroll
        for (int s = 0; s < NZ; ++s) {
            const int i = tid + NB * s;
            const int n1 = 2 * (i & (L / 2 - 1));
            const int cc = (i >> (G::logL - 1)) & (G::T - 1);
            const int pp = i >> (G::logL - 1 + G::logT);
            const floatx4 *zp = reinterpret_cast<const floatx4 *>(zb + (unsigned)(pp * (int)N + cc * L + n1));
            z[s] = a.znt ? __builtin_nontemporal_load(zp) : *zp;
        }
    };
    auto z_to_lds = [&](const floatx4 (&z)[NZ]) {
#pragma unroll
        for (int s = 0; s < NZ; ++s) {
            const int i = tid + NB * s;
            const int n1 = 2 * (i & (L / 2 - 1));
            const int cc = (i >> (G::logL - 1)) & (G::T - 1);
            const int pp = i >> (G::logL - 1 + G::logT);
            const int ad0 = G::idx(pp, cc, n1), ad1 = G::idx(pp, cc, n1 + 1);
            sre[ad0] = z[s][0];
            sim[ad0] = z[s][1];
            sre[ad1] = z[s][2];
            sim[ad1] = z[s][3];
        }
    };
    floatx4 zc[ZPRE ? NZ : 1];
    if constexpr (ZPRE) {
        if (js < je) z_loads(js, zc);
    }

    for (long long j = js; j < je; ++j) {
        // lane indices of this spectrum's iteration (see FreshIdx)
        const int tj = FreshIdx<PREC>::value ? opaque_int(tid) : tid;
        const int pol_j = tj / G::TPP, lt_j = tj % G::TPP;
        const int c_j = lt_j >> (G::logL - 4), bb_j = lt_j & (G::L16 - 1);
        const float2 *zb = a.Z + (j - a.jz0) * NPOL * N + (long long)k2_0 * L;
        if constexpr (ZPRE) {
            z_to_lds(zc);
        } else {
            // two consecutive n1 (16 bytes) per access
#pragma unroll
            for (int s = 0; s < (NPOL * G::TP) / (2 * NB); ++s) {
                const int i = tj + NB * s;
                const int n1 = 2 * (i & (L / 2 - 1));
                const int cc = (i >> (G::logL - 1)) & (G::T - 1);
                const int pp = i >> (G::logL - 1 + G::logT);
                const floatx4 *zp = reinterpret_cast<const floatx4 *>(zb + (unsigned)(pp * (int)N + cc * L + n1));
                const floatx4 z = a.znt ? __builtin_nontemporal_load(zp) : *zp;
                const int ad0 = G::idx(pp, cc, n1), ad1 = G::idx(pp, cc, n1 + 1);
                sre[ad0] = z[0];
                sim[ad0] = z[1];
                sre[ad1] = z[2];
                sim[ad1] = z[3];
            }
        }
        __syncthreads();
        if constexpr (ZPRE) {
            if (j + 1 < je) z_loads(j + 1, zc);
        }
        C v[16];
        if constexpr (F64) fft_plane<G, FftWave<G, PREC>::value, double>(sre, sim, pol_j, lt_j, a.g.tw64, v);
        else fft_plane_p<G, PREC>(sre, sim, pol_j, lt_j, a.g.tw, Wm, v, NPOL == 1);
        if constexpr (NPOL == 2) {
            if constexpr (!FftPrec<PREC>::IN_LDS) {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int ad = G::idx(pol_j, c_j, bb_j + r * G::L16);
                    sre[ad] = v[r].x;
                    sim[ad] = v[r].y;
                }
                __syncthreads();
            }
#pragma unroll
            for (int i = 0; i < BINS; ++i) {
                const int e = tj + NB * i;
                const int c = e >> G::logL, k = e & (L - 1);
                const int ax = G::idx(0, c, k), ay = G::idx(1, c, k);
                prod4(acc[i], Cx<C>::mk(sre[ax], sim[ax]), Cx<C>::mk(sre[ay], sim[ay]));
            }
            __syncthreads();
        } else {
            if constexpr (FftPrec<PREC>::IN_LDS || FftWave<G, PREC>::value) __syncthreads();
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[r][0] += (float)(v[r].x * v[r].x + v[r].y * v[r].y);
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

}  // namespace pfbs
