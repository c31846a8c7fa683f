// Auxiliary kernels of the spectrometer: dump reduction, tap-history carry,
// pre-filter test hook and the FP64 table generators; launch helpers.
#include "fft_common.h"

namespace pfbs {

hipError_t launch_front_single(const FrontArgs &a, int npol, bool pfb, int n_chunks, hipStream_t s);
hipError_t launch_front_cols(const FrontArgs &a, int npol, bool pfb, int n_chunks, hipStream_t s);
hipError_t init_single(int lds_limit);
hipError_t init_fourstep(int lds_limit);

// ------------------------------------------------------------- reduce -----

// Dump d = d_lo + blockIdx.y: carried-in sum (if the dump began in an earlier
// block) plus the chunk partials of this block in chunk order.  Complete
// dumps go to out in channel order; an incomplete one back to carried.
// Tile: 32 k2 x 32 k1 through LDS so both the partial reads (along k1) and
// the dump writes (along k2) are coalesced.  Identity order when N2 == 1.
__global__ __launch_bounds__(256) void k_reduce(ReduceArgs a) {
    __shared__ float tile[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const long long d = a.d_lo + blockIdx.y;
    const long long g_first = max(a.gid_lo, d * a.C);
    const long long g_last = min(a.gid_hi, d * a.C + a.C - 1);
    const bool carried_in = a.flush ? (a.have_carried != 0) : (d * a.n_int < a.j_lo);
    const bool complete = a.flush ? true : ((d + 1) * a.n_int <= a.j_hi);
    const long long slot = d - a.d_lo;
    const long long N = a.N;
    const bool tr = a.N2 > 1;
    long long k2b, k1b;  // tile origin
    if (tr) {
        const long long nt2 = a.N2 / 32;
        k2b = (blockIdx.x % nt2) * 32;
        k1b = (blockIdx.x / nt2) * 32;
    } else {
        k2b = 0;
        k1b = (long long)blockIdx.x * 256;
    }
    for (int q = 0; q < a.n_prod; ++q) {
        if (tr) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const long long u = (k2b + ty + 8 * i) * a.N1 + k1b + tx;
                float s = carried_in ? a.carried[q * N + u] : 0.f;
                if (!a.flush)
                    for (long long gg = g_first; gg <= g_last; ++gg)
                        s += a.part[((gg - a.gid_lo) * a.n_prod + q) * N + u];
                if (complete) tile[ty + 8 * i][tx] = s;
                else a.carried[q * N + u] = s;
            }
            if (complete) {
                __syncthreads();
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const long long k = (k2b + tx) + a.N2 * (k1b + ty + 8 * i);
                    a.out[(slot * a.n_prod + q) * N + k] = tile[tx][ty + 8 * i];
                }
                __syncthreads();
            }
        } else {
            const long long u = k1b + threadIdx.x;
            if (u < N) {
                float s = carried_in ? a.carried[q * N + u] : 0.f;
                if (!a.flush)
                    for (long long gg = g_first; gg <= g_last; ++gg)
                        s += a.part[((gg - a.gid_lo) * a.n_prod + q) * N + u];
                if (complete) a.out[(slot * a.n_prod + q) * N + u] = s;
                else a.carried[q * N + u] = s;
            }
        }
    }
}

// ------------------------------------------------------------ history -----

// dst <- the last H frames of [history | block]; frames before the stream
// start (never read) are written as zeros.
__global__ __launch_bounds__(256) void k_history(uint4 *dst, Frames fr, long long F, int H,
                                                 long long frame_vec) {
    const long long total = (long long)H * frame_vec;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
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
// Ns = r0 * 16^i (i < n16), concatenated.  FP64 sincospi, then FP32.
__global__ void k_tw16(float2 *tw, int r0, int n16) {
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
            tw[off + e] = make_float2((float)c, (float)s);
        }
        off += cnt;
        Ns *= 16;
    }
}

// Four-step twiddles: lo[m] = W_N^m (m < 2^q4), hi[m] = W_N^(m 2^q4).
__global__ void k_tw4(float2 *lo, float2 *hi, long long N, int q4) {
    const long long nlo = 1LL << q4, nhi = N >> q4;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nlo + nhi;
         e += (long long)gridDim.x * blockDim.x) {
        const long long m = e < nlo ? e : (e - nlo) << q4;
        double s, c;
        sincospi(-2.0 * (double)m / (double)N, &s, &c);
        if (e < nlo) lo[e] = make_float2((float)c, (float)s);
        else hi[e - nlo] = make_float2((float)c, (float)s);
    }
}

// ----------------------------------------------------------- launchers ----

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
    hipLaunchKernelGGL(k_tw16, dim3(64), dim3(256), 0, s, tw, 1 << (logL % 4), logL / 4);
    return hipGetLastError();
}

hipError_t launch_tables_tw4(float2 *lo, float2 *hi, long long N, int q4, hipStream_t s) {
    hipLaunchKernelGGL(k_tw4, dim3(16), dim3(256), 0, s, lo, hi, N, q4);
    return hipGetLastError();
}

size_t front_lds_bytes(const Geo &g, int npol) {
    const size_t Lp = (size_t)g.L + g.L / 16 + 1;
    return (size_t)2 * npol * g.T * Lp * sizeof(float);
}
size_t back_lds_bytes(const Geo &g, int npol) { return front_lds_bytes(g, npol); }

hipError_t launch_front(const FrontArgs &a, int npol, bool pfb, bool single, int n_chunks,
                        hipStream_t s) {
    return single ? launch_front_single(a, npol, pfb, n_chunks, s)
                  : launch_front_cols(a, npol, pfb, n_chunks, s);
}

hipError_t launch_reduce(const ReduceArgs &a, int n_dumps, hipStream_t s) {
    dim3 grid;
    if (a.N2 > 1) grid = dim3((unsigned)((a.N2 / 32) * (a.N1 / 32)), (unsigned)n_dumps);
    else grid = dim3((unsigned)((a.N + 255) / 256), (unsigned)n_dumps);
    hipLaunchKernelGGL(k_reduce, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_history(uint8_t *dst, const Frames &fr, long long F, int H, long long frame_bytes,
                          hipStream_t s) {
    const long long vec = frame_bytes / 16;
    hipLaunchKernelGGL(k_history, dim3(grid_for(H * vec, 256)), dim3(256), 0, s,
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

hipError_t kernels_init() {
    const int lim = 96 * 1024;  // largest workgroup LDS is ~74 KB
    hipError_t e = init_single(lim);
    hipError_t e2 = init_fourstep(lim);
    return e != hipSuccess ? e : e2;
}

}  // namespace pfbs
