// Auxiliary kernels of the spectrometer: dump reduction, tap-history carry,
// pre-filter test hook and the FP64 table generators; launch helpers.
#include <algorithm>

#include "fft_common.h"

namespace pfbs {

hipError_t launch_front_single(const FrontArgs &a, int npol, bool pfb, int prec, int n_chunks, hipStream_t s);
hipError_t launch_front_cols(const FrontArgs &a, int npol, bool pfb, int prec, int n_items, hipStream_t s);
hipError_t init_single(int lds_limit);
hipError_t init_fourstep(int lds_limit);

// ------------------------------------------------------------- reduce -----

// Dump d = d_lo + blockIdx.y, product q = blockIdx.z: carried-in sum (if the
// dump began in an earlier block) plus the chunk partials of this block in
// chunk order.  Complete dumps go to out in channel order; an incomplete one
// (only the last) to carried_out, a different buffer from carried_in because
// the first dump of the same launch may still be reading that one.
// Four-step order (N2 > 1): a workgroup takes 32 k2 x 32 k1, four per thread
// (reads along k1: 128-byte rows of the partials), then writes channel order
// k = k2 + N2 k1 through LDS (128-byte rows along k2).  Single pass
// (N2 == 1): 256 consecutive channels.
constexpr int kReduceTile = 32;

// s[e] = carried-in value (if any) + the chunk partials in chunk order, for NE
// elements at offsets u[e]; the elements' loads go out together (eight chunks
// at a time) so that one thread keeps 8*NE loads in flight.
template <int NE>
__device__ __forceinline__ void reduce_sums(const ReduceArgs &a, int q, bool carried_in, long long g_first,
                                            long long g_last, const long long (&u)[NE], float (&s)[NE]) {
    const long long N = a.N;
#pragma unroll
    for (int e = 0; e < NE; ++e) s[e] = carried_in ? a.carried_in[q * N + u[e]] : 0.f;
    if (a.flush) return;
    const long long stride = (long long)a.n_prod * N;
    const float *pp = a.part + q * N;
    long long gg = g_first;
    for (; gg + 8 <= g_last + 1; gg += 8) {
        float v[8][NE];
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
            for (int e = 0; e < NE; ++e) v[i][e] = pp[(gg + i - a.gid_lo) * stride + u[e]];
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
            for (int e = 0; e < NE; ++e) s[e] += v[i][e];
    }
    for (; gg <= g_last; ++gg)
#pragma unroll
        for (int e = 0; e < NE; ++e) s[e] += pp[(gg - a.gid_lo) * stride + u[e]];
}

__device__ void reduce_body(const ReduceArgs &a, int bx, int by, int bz) {
    __shared__ float tile[kReduceTile][kReduceTile + 1];
    constexpr int R = kReduceTile * kReduceTile / 256;  // elements per thread (four-step)
    const int t = threadIdx.x;
    const long long d = a.d_lo + by;
    const int q = bz;
    const long long g_first = max(a.gid_lo, d * a.C);
    const long long g_last = min(a.gid_hi, d * a.C + a.C - 1);
    const bool carried_in = a.flush ? (a.have_carried != 0) : (d * a.n_int < a.j_lo);
    const bool complete = a.flush ? true : ((d + 1) * a.n_int <= a.j_hi);
    const long long slot = d - a.d_lo;
    const long long N = a.N;
    float *out = a.out + (slot * a.n_prod + q) * N;
    if (a.N2 > 1) {
        const long long nt2 = a.N2 / kReduceTile;
        const long long k2b = (bx % nt2) * kReduceTile, k1b = (bx / nt2) * kReduceTile;
        long long u[R];
        float sv[R];
#pragma unroll
        for (int e = 0; e < R; ++e) u[e] = (k2b + (t >> 5) + 8 * e) * a.N1 + k1b + (t & 31);
        reduce_sums<R>(a, q, carried_in, g_first, g_last, u, sv);
        if (!complete) {
#pragma unroll
            for (int e = 0; e < R; ++e) a.carried_out[q * N + u[e]] = sv[e];
            return;
        }
#pragma unroll
        for (int e = 0; e < R; ++e) tile[(t >> 5) + 8 * e][t & 31] = sv[e];
        __syncthreads();
#pragma unroll
        for (int e = 0; e < R; ++e) {
            const int dk2 = t & 31, dk1 = (t >> 5) + 8 * e;
            out[(k2b + dk2) + a.N2 * (k1b + dk1)] = tile[dk2][dk1];
        }
    } else {
        const long long u0 = (long long)bx * 256 + t;
        if (u0 >= N) return;
        const long long u[1] = {u0};
        float sv[1];
        reduce_sums<1>(a, q, carried_in, g_first, g_last, u, sv);
        if (!complete) a.carried_out[q * N + u0] = sv[0];
        else out[u0] = sv[0];
    }
}

// grid.y is capped at 65535: a workgroup row walks dumps y, y + gridDim.y, ...
__global__ __launch_bounds__(256) void k_reduce(ReduceArgs a, int n_dumps) {
    for (int by = blockIdx.y; by < n_dumps; by += gridDim.y) {
        reduce_body(a, blockIdx.x, by, blockIdx.z);
        __syncthreads();  // the LDS tile is reused by the next dump
    }
}

// ---------------------------------------------------------- dump form -----

// Dump row y (blockIdx.y), channel pair (k, k + N/2) per thread, in place:
// the four products of a channel become I = XX + YY, Q = XX - YY,
// U = 2 Re XY*, V = -2 Im XY* (stokes), and channel k moves to position
// (k + N/2) mod N (shift), i.e. the two halves of the row swap.
__global__ __launch_bounds__(256) void k_dump_format(float *out, long long n_dumps, long long N, int n_prod,
                                                     int stokes, int shift) {
    const long long h = N / 2;
    const long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (k >= h) return;
    for (long long y = blockIdx.y; y < n_dumps; y += gridDim.y) {
    float *row = out + y * n_prod * N;
    float a[4], b[4];
    for (int q = 0; q < n_prod; ++q) {
        a[q] = row[q * N + k];
        b[q] = row[q * N + k + h];
    }
    if (stokes) {
        const float ai = a[0] + a[1], aq = a[0] - a[1], au = 2.f * a[2], av = -2.f * a[3];
        const float bi = b[0] + b[1], bq = b[0] - b[1], bu = 2.f * b[2], bv = -2.f * b[3];
        a[0] = ai; a[1] = aq; a[2] = au; a[3] = av;
        b[0] = bi; b[1] = bq; b[2] = bu; b[3] = bv;
    }
    for (int q = 0; q < n_prod; ++q) {
        row[q * N + k] = shift ? b[q] : a[q];
        row[q * N + k + h] = shift ? a[q] : b[q];
    }
    }
}

// ------------------------------------------------------------ history -----

// dst <- the last H frames of [history | block]; frames before the stream
// start (never read) are written as zeros.
__device__ void history_body(uint4 *dst, const Frames &fr, long long F, int H, long long frame_vec,
                             int bid, int nblk) {
    const long long total = (long long)H * frame_vec;
    for (long long i = bid * (long long)blockDim.x + threadIdx.x; i < total;
         i += (long long)nblk * blockDim.x) {
        const long long fp = i / frame_vec, off = i - fp * frame_vec;
        const long long gidx = fr.fs + F - H + fp;  // global frame index
        uint4 v = make_uint4(0, 0, 0, 0);
        if (gidx >= fr.fs)
            v = reinterpret_cast<const uint4 *>(fr.blk)[(gidx - fr.fs) * frame_vec + off];
        else if (gidx >= fr.hf0 && gidx >= 0)
            v = reinterpret_cast<const uint4 *>(fr.hist)[(gidx - fr.hf0) * frame_vec + off];
        dst[i] = v;
    }
}

__global__ __launch_bounds__(256) void k_history(uint4 *dst, Frames fr, long long F, int H,
                                                 long long frame_vec) {
    history_body(dst, fr, F, H, frame_vec, blockIdx.x, gridDim.x);
}

// A plan's tail in one launch: the dump reduction on the first blocks and the
// tap-history copy on the rest (they touch disjoint buffers: the history is
// written to the buffer the next block reads, the reduction reads partial
// sums and writes dumps and carried sums).
__global__ __launch_bounds__(256) void k_reduce_history(ReduceArgs a, int gx, int n_dumps, uint4 *hdst, Frames fr,
                                                        long long F, int H, long long frame_vec, int n_hist) {
    const int n_red = gx * n_dumps * a.n_prod;
    const int b = blockIdx.x;
    if (b < n_red) {
        const int per_z = gx * n_dumps;
        const int bz = b / per_z, rem = b - bz * per_z;
        reduce_body(a, rem % gx, rem / gx, bz);
    } else {
        history_body(hdst, fr, F, H, frame_vec, b - n_red, n_hist);
    }
}

// Batched tail: dump reductions and tap-history copies of every sub-band.
__global__ __launch_bounds__(256) void k_batch_tail(const BatchTailEntry *__restrict__ t, int n) {
    if (n <= 0) return;
    int e = 0;
    while (e + 1 < n && (int)blockIdx.x >= t[e + 1].wg0) ++e;
    const int vb = blockIdx.x - t[e].wg0;
    if (vb < 0 || vb >= t[e].wgn) return;
    BatchTailEntry E = t[e];  // private copy, as in the batched FFT kernels
    globalise(E.r);
    globalise(E.fr);
    E.hdst = as_global(E.hdst);
    if (E.kind == 0) {
        const int per_z = E.gx * E.gy;
        const int bz = vb / per_z, rem = vb - bz * per_z;
        reduce_body(E.r, rem % E.gx, rem / E.gx, bz);
    } else {
        history_body(reinterpret_cast<uint4 *>(E.hdst), E.fr, E.F, E.H, E.frame_vec, vb, E.wgn);
    }
}

// ---------------------------------------------------------- debug PFB -----

// y[(j - j_lo)][pol][n][2] for spectra [j_lo, j_hi): the pre-filter exactly as
// the FFT kernels compute it (same tap order and fused multiply-adds).
template <int NPOL, bool PFB>
__global__ __launch_bounds__(256) void k_debug_pfb(float *y, Frames fr, const float *taps, long long N,
                                                   int P, long long j_lo, long long j_hi) {
    typedef typename Sample<NPOL>::word W;
    const long long total = (j_hi - j_lo) * N;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        const long long jr = i / N, n = i - jr * N;
        const long long j = j_lo + jr;
        float2 acc[NPOL];
#pragma unroll
        for (int pol = 0; pol < NPOL; ++pol) acc[pol] = make_float2(0.f, 0.f);
        const int PP = PFB ? P : 1;
        for (int p = 0; p < PP; ++p) {
            const W w = frame_ptr<NPOL>(fr, j + p, N)[n];
            if (PFB) tap_fma<NPOL>(acc, taps[p * N + n], w);
            else Sample<NPOL>::unpack(w, acc);
        }
#pragma unroll
        for (int pol = 0; pol < NPOL; ++pol) {
            y[((jr * NPOL + pol) * N + n) * 2 + 0] = acc[pol].x;
            y[((jr * NPOL + pol) * N + n) * 2 + 1] = acc[pol].y;
        }
    }
}

// ------------------------------------------------------------- tables -----

// Filter taps, evaluated in FP64 on the device and rounded once to FP32.
__global__ void k_taps(float *h, long long N, int P, int window, const double *custom) {
    const long long L = N * P;
    for (long long m = blockIdx.x * (long long)blockDim.x + threadIdx.x; m < L;
         m += (long long)gridDim.x * blockDim.x) {
        double v;
        if (window == 1) {
            v = 1.0;
        } else if (window == 2) {
            v = custom[m];
        } else {
            const double u = (double)(m - L / 2) / (double)N;
            const double s = (m == L / 2) ? 1.0 : sinpi(u) / (3.14159265358979323846 * u);
            const double w = 0.5 - 0.5 * cospi(2.0 * (double)m / (double)L);
            v = s * w;
        }
        h[m] = (float)v;
    }
}

// Radix-16 pass twiddles W_(16 Ns)^(k r), k < Ns, r = 1..15, for the passes
// Ns = r0 * 16^i (i < n16), concatenated.  FP64 sincospi, then rounded to
// the table's type (float2, or kept in FP64 for the FP64 row pass).
template <class C>
__global__ void k_tw16(C *tw, int r0, int n16) {
    long long off = 0;
    long long Ns = r0;
    for (int i = 0; i < n16; ++i) {
        const long long cnt = Ns * 15;
        for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < cnt;
             e += (long long)gridDim.x * blockDim.x) {
            const long long k = e / 15, r = e % 15 + 1;
            const long long M = 16 * Ns;
            const long long kr = (k * r) % M;
            double s, c;
            sincospi(-2.0 * (double)kr / (double)M, &s, &c);
            if constexpr (sizeof(C) == sizeof(float2)) tw[off + e] = make_float2((float)c, (float)s);
            else tw[off + e] = make_double2(c, s);
        }
        off += cnt;
        Ns *= 16;
    }
}

// Matrix-core operands of the radix-16 DFT (hi and lo FP16 parts of its real
// form, from FP64), one row of four 16-byte values per lane.
__global__ void k_mfma_w(uint4 *mw) {
    const int lane = threadIdx.x;
    const MfmaW w = mfma_dft16_operands(lane);
    mw[lane * 4 + 0] = __builtin_bit_cast(uint4, w.hr);
    mw[lane * 4 + 1] = __builtin_bit_cast(uint4, w.hi);
    mw[lane * 4 + 2] = __builtin_bit_cast(uint4, w.lr);
    mw[lane * 4 + 3] = __builtin_bit_cast(uint4, w.li);
}

// Four-step twiddles tw4[n1*N2 + k2] = W_N^(n1 k2), FP64 sincospi then FP32.
__global__ void k_tw4(float2 *tw4, long long N1, long long N2) {
    const long long N = N1 * N2;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < N;
         e += (long long)gridDim.x * blockDim.x) {
        const long long n1 = e / N2, k2 = e - n1 * N2;
        const long long m = (n1 * k2) % N;
        double s, c;
        sincospi(-2.0 * (double)m / (double)N, &s, &c);
        tw4[e] = make_float2((float)c, (float)s);
    }
}

// Synthetic int8 words for the autotuner: each byte a hashed function of its
// index (finaliser of MurmurHash3), folded to roughly Gaussian-sized values.
__global__ void k_synth(uint32_t *w, long long n, uint32_t seed) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        uint32_t x = (uint32_t)i * 0x9E3779B9u ^ seed;
        x ^= x >> 16; x *= 0x85EBCA6Bu; x ^= x >> 13; x *= 0xC2B2AE35u; x ^= x >> 16;
        // each byte: sum of two 5-bit fields minus 31 -> [-31, 31], triangular
        uint32_t o = 0;
        for (int b = 0; b < 4; ++b) {
            const uint32_t y = (x >> (8 * b)) * 0x2545F491u;
            const int v = (int)((y >> 5) & 31) + (int)((y >> 11) & 31) - 31;
            o |= (uint32_t)(uint8_t)(int8_t)v << (8 * b);
        }
        w[i] = o;
    }
}

// ----------------------------------------------------------- launchers ----

hipError_t launch_synth(uint32_t *words, long long n_words, uint32_t seed, hipStream_t s) {
    hipLaunchKernelGGL(k_synth, dim3(1024), dim3(256), 0, s, words, n_words, seed);
    return hipGetLastError();
}


static int grid_for(long long n, int per_block) {
    long long b = (n + per_block - 1) / per_block;
    if (b < 1) b = 1;
    if (b > 65536) b = 65536;
    return (int)b;
}

hipError_t launch_tables_taps(float *h, long long N, int P, int window, const double *d_custom,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_taps, dim3(grid_for(N * P, 256)), dim3(256), 0, s, h, N, P, window,
                       d_custom);
    return hipGetLastError();
}

hipError_t launch_tables_tw16(float2 *tw, int L, hipStream_t s) {
    const int logL = ilog2c(L);
    hipLaunchKernelGGL(k_tw16<float2>, dim3(64), dim3(256), 0, s, tw, 1 << (logL % 4), logL / 4);
    return hipGetLastError();
}

hipError_t launch_tables_mfma(uint4 *mw, hipStream_t s) {
    hipLaunchKernelGGL(k_mfma_w, dim3(1), dim3(64), 0, s, mw);
    return hipGetLastError();
}

hipError_t launch_tables_tw16_f64(double2 *tw, int L, hipStream_t s) {
    const int logL = ilog2c(L);
    hipLaunchKernelGGL(k_tw16<double2>, dim3(64), dim3(256), 0, s, tw, 1 << (logL % 4), logL / 4);
    return hipGetLastError();
}

hipError_t launch_tables_tw4(float2 *tw4, long long N1, long long N2, hipStream_t s) {
    hipLaunchKernelGGL(k_tw4, dim3(grid_for(N1 * N2, 256)), dim3(256), 0, s, tw4, N1, N2);
    return hipGetLastError();
}

size_t front_lds_bytes(const Geo &g, int npol) {
    const size_t Lp = (size_t)lds_pitch(g.L);
    return (size_t)2 * npol * g.T * Lp * sizeof(float);
}
// The FP64 row pass (prec 3) keeps double planes.
size_t back_lds_bytes(const Geo &g, int npol, int prec) {
    return front_lds_bytes(g, npol) * (prec == 3 ? 2 : 1);
}

hipError_t launch_front(const FrontArgs &a, int npol, bool pfb, bool single, int prec, int n_items,
                        hipStream_t s) {
    return single ? launch_front_single(a, npol, pfb, prec, n_items, s)
                  : launch_front_cols(a, npol, pfb, prec, n_items, s);
}

hipError_t launch_reduce(const ReduceArgs &a, int n_dumps, hipStream_t s) {
    if (n_dumps <= 0) return hipSuccess;
    const unsigned gy = (unsigned)std::min(n_dumps, 65535);
    dim3 grid;
    if (a.N2 > 1) grid = dim3((unsigned)((a.N2 / kReduceTile) * (a.N1 / kReduceTile)), gy, (unsigned)a.n_prod);
    else grid = dim3((unsigned)((a.N + 255) / 256), gy, (unsigned)a.n_prod);
    PFBS_LAUNCH(k_reduce, grid, dim3(256), 0, s, a, n_dumps);
    return hipGetLastError();
}

hipError_t launch_reduce_history(const ReduceArgs &a, int n_dumps, uint8_t *dst, const Frames &fr, long long F,
                                 int H, long long frame_bytes, hipStream_t s) {
    const int gx = a.N2 > 1 ? (int)((a.N2 / kReduceTile) * (a.N1 / kReduceTile)) : (int)((a.N + 255) / 256);
    const long long vec = frame_bytes / 16;
    const int n_hist = grid_for(H * vec, 256);
    const long long n_red = (long long)gx * std::max(n_dumps, 0) * a.n_prod;
    if (n_red + n_hist > 0x7fffffffLL) return hipErrorInvalidValue;
    PFBS_LAUNCH(k_reduce_history, dim3((unsigned)(n_red + n_hist)), dim3(256), 0, s, a, gx, std::max(n_dumps, 0),
                reinterpret_cast<uint4 *>(dst), fr, F, H, vec, n_hist);
    return hipGetLastError();
}

hipError_t launch_dump_format(float *out, long long n_dumps, long long N, int n_prod, int stokes, int shift,
                              hipStream_t s) {
    if (n_dumps <= 0) return hipSuccess;
    if ((stokes && n_prod != 4) || N < 2) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((N / 2 + 255) / 256), (unsigned)std::min<long long>(n_dumps, 65535));
    PFBS_LAUNCH(k_dump_format, grid, dim3(256), 0, s, out, n_dumps, N, n_prod, stokes, shift);
    return hipGetLastError();
}

hipError_t launch_history(uint8_t *dst, const Frames &fr, long long F, int H, long long frame_bytes,
                          hipStream_t s) {
    const long long vec = frame_bytes / 16;
    PFBS_LAUNCH(k_history, dim3(grid_for(H * vec, 256)), dim3(256), 0, s,
                       reinterpret_cast<uint4 *>(dst), fr, F, H, vec);
    return hipGetLastError();
}

hipError_t launch_debug_pfb(float *y, const Frames &fr, const float *taps, long long N, int P,
                            int npol, bool pfb, long long j_lo, long long j_hi, hipStream_t s) {
    const dim3 grid(grid_for((j_hi - j_lo) * N, 256)), block(256);
    if (npol == 2) {
        if (pfb) hipLaunchKernelGGL((k_debug_pfb<2, true>), grid, block, 0, s, y, fr, taps, N, P, j_lo, j_hi);
        else hipLaunchKernelGGL((k_debug_pfb<2, false>), grid, block, 0, s, y, fr, taps, N, P, j_lo, j_hi);
    } else {
        if (pfb) hipLaunchKernelGGL((k_debug_pfb<1, true>), grid, block, 0, s, y, fr, taps, N, P, j_lo, j_hi);
        else hipLaunchKernelGGL((k_debug_pfb<1, false>), grid, block, 0, s, y, fr, taps, N, P, j_lo, j_hi);
    }
    return hipGetLastError();
}

const void *batch_tail_fn() { return reinterpret_cast<const void *>(&k_batch_tail); }

hipError_t kernels_init() {
    const int lim = 96 * 1024;  // largest workgroup LDS is ~74 KB
    hipError_t e = init_single(lim);
    hipError_t e2 = init_fourstep(lim);
    return e != hipSuccess ? e : e2;
}

}  // namespace pfbs
