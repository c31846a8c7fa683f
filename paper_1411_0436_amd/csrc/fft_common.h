// Device building blocks shared by the FFT kernels: complex arithmetic, the
// radix-2/4/8/16 DFTs, the compile-time sub-FFT geometry, the Stockham passes
// in LDS, int8 unpacking and the polarisation products.
#pragma once

#include <type_traits>

#include "pfbs_internal.h"

namespace pfbs {

constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v >> 1); }

// A pointer read from device memory is a generic (flat) address to the
// compiler, and accesses through it become flat loads and stores, which take
// the LDS/scratch aperture checks.  Every buffer of this library is global
// device memory; passing the address through an integer into the global
// address space lets the compiler emit global loads and stores instead.
template <class T>
__device__ __forceinline__ T *as_global(T *p) {
    return (T *)(__attribute__((address_space(1))) T *)(unsigned long long)p;
}

__device__ __forceinline__ void globalise(Frames &f) {
    f.blk = as_global(f.blk);
    f.hist = as_global(f.hist);
}
__device__ __forceinline__ void globalise(FrontArgs &a) {
    globalise(a.fr);
    a.taps = as_global(a.taps);
    a.g.tw = as_global(a.g.tw);
    a.Z = as_global(a.Z);
    a.tw4 = as_global(a.tw4);
    a.part = as_global(a.part);
}
__device__ __forceinline__ void globalise(BackArgs &a) {
    a.Z = as_global(a.Z);
    a.g.tw = as_global(a.g.tw);
    a.part = as_global(a.part);
}
__device__ __forceinline__ void globalise(ReduceArgs &a) {
    a.part = as_global(a.part);
    a.carried_in = as_global(a.carried_in);
    a.carried_out = as_global(a.carried_out);
    a.out = as_global(a.out);
}

// Raw buffer loads: a wave-uniform base and size in a scalar resource
// descriptor and a 32-bit per-lane byte offset (a frame or a tap row is at
// most 4 MB), so a load needs one vector register for its address instead of
// a 64-bit pair, and loads past `bytes` return zero instead of touching
// memory.  Word 3 of the descriptor: 32-bit data format, as raw loads
// require on this architecture.
typedef __amdgpu_buffer_rsrc_t Rsrc;
__device__ __forceinline__ Rsrc make_rsrc(const void *base, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}
template <class T> __device__ __forceinline__ T buf_load(Rsrc r, unsigned off);
template <> __device__ __forceinline__ uint4 buf_load<uint4>(Rsrc r, unsigned off) {
    return __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}
template <> __device__ __forceinline__ float4 buf_load<float4>(Rsrc r, unsigned off) {
    return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}
template <> __device__ __forceinline__ uint2 buf_load<uint2>(Rsrc r, unsigned off) {
    return __builtin_bit_cast(uint2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}

// --------------------------------------------------------------- complex --

// Complex values of the FFT passes: float2 (FP32 arithmetic) or double2 (the
// FP64 row pass).  Cx<C> gives the real type, a constructor and the DFT
// constants in that precision.
template <class C> struct Cx;
template <> struct Cx<float2> {
    typedef float R;
    __device__ __forceinline__ static float2 mk(float a, float b) { return make_float2(a, b); }
    static constexpr float c1 = 0.92387953251128675613f, s1 = 0.38268343236508977173f;  // cos, sin(pi/8)
    static constexpr float h = 0.70710678118654752440f;                                   // cos(pi/4)
};
template <> struct Cx<double2> {
    typedef double R;
    __device__ __forceinline__ static double2 mk(double a, double b) { return make_double2(a, b); }
    static constexpr double c1 = 0.92387953251128675613, s1 = 0.38268343236508977173;
    static constexpr double h = 0.70710678118654752440;
};
// Element type of an LDS plane -> its complex type.
template <class T> struct Cplx;
template <> struct Cplx<float> { typedef float2 type; };
template <> struct Cplx<double> { typedef double2 type; };

template <class C> __device__ __forceinline__ C cadd(C a, C b) { return Cx<C>::mk(a.x + b.x, a.y + b.y); }
template <class C> __device__ __forceinline__ C csub(C a, C b) { return Cx<C>::mk(a.x - b.x, a.y - b.y); }
template <class C> __device__ __forceinline__ C cmul(C a, C w) {
    return Cx<C>::mk(a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x);
}
template <class C> __device__ __forceinline__ C mul_mi(C a) { return Cx<C>::mk(a.y, -a.x); }  // a * (-i)

// Forward DFTs (kernel e^{-2 pi i k n / R}), natural order in and out.
template <class C> __device__ __forceinline__ void dft4(C &a0, C &a1, C &a2, C &a3) {
    C t0 = cadd(a0, a2), t1 = csub(a0, a2);
    C t2 = cadd(a1, a3), t3 = mul_mi(csub(a1, a3));
    a0 = cadd(t0, t2);
    a2 = csub(t0, t2);
    a1 = cadd(t1, t3);
    a3 = csub(t1, t3);
}

template <class C> __device__ __forceinline__ void dft2(C *v) {
    C a = v[0];
    v[0] = cadd(a, v[1]);
    v[1] = csub(a, v[1]);
}

// 8 = 2 x 4: n = m + 2r, k = q + 4s.
template <class C> __device__ __forceinline__ void dft8(C *v) {
    typedef typename Cx<C>::R R;
    const R h = Cx<C>::h;
    C e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    C o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4(e0, e1, e2, e3);
    dft4(o0, o1, o2, o3);
    o1 = Cx<C>::mk((o1.x + o1.y) * h, (o1.y - o1.x) * h);   // * W8^1
    o2 = mul_mi(o2);                                        // * W8^2
    o3 = Cx<C>::mk((o3.y - o3.x) * h, -(o3.x + o3.y) * h);  // * W8^3
    v[0] = cadd(e0, o0); v[4] = csub(e0, o0);
    v[1] = cadd(e1, o1); v[5] = csub(e1, o1);
    v[2] = cadd(e2, o2); v[6] = csub(e2, o2);
    v[3] = cadd(e3, o3); v[7] = csub(e3, o3);
}

// 16 = 4 x 4: n = m + 4r, k = q + 4s; inner twiddle W16^(m q).
template <class C> __device__ __forceinline__ void dft16(C *v) {
    typedef typename Cx<C>::R R;
    const R c1 = Cx<C>::c1, s1 = Cx<C>::s1, h = Cx<C>::h;
    C u[16];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        C a0 = v[m], a1 = v[m + 4], a2 = v[m + 8], a3 = v[m + 12];
        dft4(a0, a1, a2, a3);
        u[m * 4 + 0] = a0; u[m * 4 + 1] = a1; u[m * 4 + 2] = a2; u[m * 4 + 3] = a3;
    }
    u[5] = cmul(u[5], Cx<C>::mk(c1, -s1));                                 // W^1
    u[6] = Cx<C>::mk((u[6].x + u[6].y) * h, (u[6].y - u[6].x) * h);        // W^2
    u[7] = cmul(u[7], Cx<C>::mk(s1, -c1));                                 // W^3
    u[9] = Cx<C>::mk((u[9].x + u[9].y) * h, (u[9].y - u[9].x) * h);        // W^2
    u[10] = mul_mi(u[10]);                                                 // W^4
    u[11] = Cx<C>::mk((u[11].y - u[11].x) * h, -(u[11].x + u[11].y) * h);  // W^6
    u[13] = cmul(u[13], Cx<C>::mk(s1, -c1));                               // W^3
    u[14] = Cx<C>::mk((u[14].y - u[14].x) * h, -(u[14].x + u[14].y) * h);  // W^6
    u[15] = cmul(u[15], Cx<C>::mk(-c1, s1));                               // W^9
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        C b0 = u[q], b1 = u[4 + q], b2 = u[8 + q], b3 = u[12 + q];
        dft4(b0, b1, b2, b3);
        v[q] = b0; v[q + 4] = b1; v[q + 8] = b2; v[q + 12] = b3;
    }
}

template <int R, class C> __device__ __forceinline__ void dftR(C *v) {
    if constexpr (R == 2) dft2(v);
    else if constexpr (R == 4) dft4(v[0], v[1], v[2], v[3]);
    else dft8(v);
}

// -------------------------------------------------------------- geometry --

// Batched sub-FFT of length L = r0 * 16^n16 over T = TP/L columns per
// polarisation (TP complex points per polarisation per workgroup step, done by
// TPP = TP/16 threads, each owning one radix-16 butterfly).  LDS: re and im
// planes [pol][c][Lp], element e of a column at e + (e >> PS) (one pad word
// per 2^PS) and one more pad word per column.  The 32 four-byte banks serve a
// wave's access in two halves of 32 lanes, and no single padding makes every
// access pattern of a kernel conflict-free: PS = 4 suits the column pass, PS
// = 5 measured faster in the single-pass and most row-pass kernels.  The
// host sizes LDS for PS = 4, which is the larger.
template <int L_, int TP_ = kTilePoints, int PS_ = 4>
struct Geom {
    static constexpr int L = L_;
    static constexpr int TP = TP_;
    static constexpr int PS = PS_;
    static constexpr int TPP = TP / 16;   // threads per polarisation
    static constexpr int logL = ilog2c(L);
    static constexpr int T = TP / L;
    static constexpr int logT = ilog2c(T);
    static constexpr int n16 = logL / 4;
    static constexpr int r0 = 1 << (logL % 4);
    static constexpr int L16 = L / 16;
    static constexpr int Lp = L + (L >> PS) + 1;
    static constexpr int plane = T * Lp;  // floats of one polarisation plane
    static_assert(T >= 1 && L >= 16, "sub-FFT geometry");
    static_assert((PS == 4 || PS == 5) && Lp <= lds_pitch(L), "LDS padding within the host's LDS size");
    // every column is transformed by lanes of a single wave
    static constexpr bool WAVE_COLS = L16 <= 64 && TPP % 64 == 0;
    __host__ __device__ __forceinline__ static constexpr int idx(int pol, int c, int e) {
        return (pol * T + c) * Lp + e + (e >> PS);
    }
    // Offset of radix-16 pass i in the twiddle table (Ns = r0 * 16^i entries each of 15).
    static constexpr int tw_off(int i) { return i == 0 ? 0 : tw_off(i - 1) + r0 * (1 << (4 * (i - 1))) * 15; }
};

// Synchronisation between the passes of a sub-FFT: a workgroup barrier, or,
// where the lanes of one wave transform each column alone (WAVE), a fence
// that only keeps the compiler from moving LDS accesses across it: the LDS
// performs one wave's accesses in program order.
template <bool WAVE>
__device__ __forceinline__ void pass_sync() {
    if constexpr (WAVE) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// First pass, radix R in {2,4,8}, sub-transform size 1 (no twiddle).  Thread
// lt (0..TPP-1) of polarisation pol does 16/R butterflies: with WAVE, those of
// its own column of the radix-16 passes (bb + s*L/16), else bb + s*TPP
// counted across the columns.
template <class G, int R, bool WAVE, class T = float>
__device__ __forceinline__ void pass_small(T *sre, T *sim, int pol, int lt) {
    typedef typename Cplx<T>::type C;
    constexpr int PER = 16 / R;
    constexpr int logLR = G::logL - ilog2c(R);
    constexpr int LR = 1 << logLR;
    auto butterfly = [&](int s, int &c, int &bb) {
        if constexpr (WAVE) {
            c = lt >> (G::logL - 4);
            bb = (lt & (G::L16 - 1)) + s * G::L16;
        } else {
            const int b = lt + s * G::TPP;
            c = b >> logLR;
            bb = b & (LR - 1);
        }
    };
    C v[PER][R];
#pragma unroll
    for (int s = 0; s < PER; ++s) {
        int c, bb;
        butterfly(s, c, bb);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int a = G::idx(pol, c, bb + r * LR);
            v[s][r] = Cx<C>::mk(sre[a], sim[a]);
        }
    }
    pass_sync<WAVE>();
#pragma unroll
    for (int s = 0; s < PER; ++s) {
        int c, bb;
        butterfly(s, c, bb);
        dftR<R>(v[s]);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int a = G::idx(pol, c, bb * R + r);
            sre[a] = v[s][r].x;
            sim[a] = v[s][r].y;
        }
    }
    pass_sync<WAVE>();
}

// Radix-16 pass i (sub-transform size Ns = r0*16^i): butterfly bb of column c
// reads elements bb + r*L/16, applies W_(16 Ns)^(k r) with k = bb mod Ns, and
// (except in the last pass) writes element (bb-k)*16 + k + r*Ns.  With WAVE
// the last pass ends without a barrier.
template <class G, int I, bool WAVE, class T = float>
__device__ __forceinline__ void pass16(T *sre, T *sim, int pol, int lt, const typename Cplx<T>::type *tw,
                                       typename Cplx<T>::type (&v)[16]) {
    typedef typename Cplx<T>::type C;
    constexpr int Ns = G::r0 * (1 << (4 * I));
    constexpr bool LAST = I == G::n16 - 1;
    const int c = lt >> (G::logL - 4), bb = lt & (G::L16 - 1);
    const int k = bb & (Ns - 1);
    C w[16];
    if (Ns > 1) {
        const C *t = tw + G::tw_off(I) + k * 15;
#pragma unroll
        for (int r = 1; r < 16; ++r) w[r] = t[r - 1];
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int a = G::idx(pol, c, bb + r * G::L16);
        v[r] = Cx<C>::mk(sre[a], sim[a]);
    }
    if (!(WAVE && LAST)) pass_sync<WAVE>();
    if (Ns > 1) {
#pragma unroll
        for (int r = 1; r < 16; ++r) v[r] = cmul(v[r], w[r]);
    }
    dft16(v);
    if (!LAST) {
        const int base = ((bb - k) << 4) + k;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int a = G::idx(pol, c, base + r * Ns);
            sre[a] = v[r].x;
            sim[a] = v[r].y;
        }
        pass_sync<WAVE>();
    }
}

template <class G, int I, bool WAVE, class T = float>
__device__ __forceinline__ void passes16(T *sre, T *sim, int pol, int lt, const typename Cplx<T>::type *tw,
                                         typename Cplx<T>::type (&v)[16]) {
    pass16<G, I, WAVE, T>(sre, sim, pol, lt, tw, v);
    if constexpr (I + 1 < G::n16) passes16<G, I + 1, WAVE, T>(sre, sim, pol, lt, tw, v);
}

// Whole batched FFT of the columns of one polarisation plane held in LDS.
// On return thread lt holds X_c[bb + r*L/16], r = 0..15, with
// c = lt / (L/16), bb = lt mod (L/16).  Every thread of the workgroup must
// call it.  Without WAVE it contains workgroup barriers and ends with one;
// with WAVE (G::WAVE_COLS) the passes synchronise within each wave only, and
// on return other waves may still be reading the plane: a thread may then
// overwrite only the positions it holds in v until a workgroup barrier.
template <class G, bool WAVE = false, class T = float>
__device__ __forceinline__ void fft_plane(T *sre, T *sim, int pol, int lt, const typename Cplx<T>::type *tw,
                                          typename Cplx<T>::type (&v)[16]) {
    static_assert(!WAVE || G::WAVE_COLS, "wave-local passes need columns within one wave");
    if constexpr (G::r0 > 1) pass_small<G, G::r0, WAVE, T>(sre, sim, pol, lt);
    passes16<G, 0, WAVE, T>(sre, sim, pol, lt, tw, v);
}

// ------------------------------------------------- matrix-core radix 16 --
//
// A radix-16 pass as a dense product on the FP16 matrix cores
// (v_mfma_f32_16x16x32_f16, FP32 accumulation).  One wave transforms 16
// butterflies at a time: Y = W16 * X with the complex 16x16 DFT matrix in its
// real 16x32 form, rows Re Y (operand ar) and Im Y (operand ai), columns
// k = 2r + c for input point r and component c (0 = re, 1 = im):
//   ar[m][2r] = Re W[m][r], ar[m][2r+1] = -Im W[m][r],
//   ai[m][2r] = Im W[m][r], ai[m][2r+1] =  Re W[m][r].
// Lane l holds butterfly n = l mod 16 and its input points 4(l/16)..+3 (the
// B-operand layout of this instruction), so it can apply the pass twiddles
// itself, and receives the outputs 4(l/16)..+3 of the same butterfly (the
// accumulator layout).  Each butterfly's inputs are scaled by a power of two
// that puts their largest component just below 2^15, then rounded to
// FP16.  MFMA_FP16 uses single FP16 values of the matrix and of the data (one
// product, relative rounding 2^-11 per operand); MFMA_FP16X2 splits both into
// hi + lo pairs (x = hi + lo + O(2^-22 x)) and sums Wlo*hi + Whi*lo + Whi*hi.
// The scale is undone exactly on the FP32 outputs.
typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef _Float16 half2v __attribute__((ext_vector_type(2)));
typedef float float2v __attribute__((ext_vector_type(2)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

struct MfmaW {
    half8 hr, hi, lr, li;   // hi and lo parts of the Re-row and Im-row operands
};

// Operands of lane `lane`, from W16^e = cos(pi e/8) - i sin(pi e/8) in double
// (run once per plan by the table kernel; the FFT kernels load the result).
__device__ __forceinline__ MfmaW mfma_dft16_operands(int lane) {
    const int m = lane & 15, kb = lane >> 4;
    MfmaW w;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int r = 4 * kb + (j >> 1);
        const int e = (m * r) & 15;
        double sn, cs;
        sincospi((double)e / 8.0, &sn, &cs);
        const double wr = cs, wi = -sn;
        const double vr = (j & 1) ? -wi : wr;
        const double vi = (j & 1) ? wr : wi;
        const _Float16 hr = (_Float16)vr, hi = (_Float16)vi;
        w.hr[j] = hr;
        w.hi[j] = hi;
        w.lr[j] = (_Float16)(vr - (double)hr);
        w.li[j] = (_Float16)(vi - (double)hi);
    }
    return w;
}

// The operands of lane `lane` from the plan's table: uint4 [64 lanes][4]
// holding hr, hi, lr, li.
__device__ __forceinline__ MfmaW mfma_operands_load(const uint4 *t, int lane) {
    MfmaW w;
    const uint4 *q = t + lane * 4;
    w.hr = __builtin_bit_cast(half8, q[0]);
    w.hi = __builtin_bit_cast(half8, q[1]);
    w.lr = __builtin_bit_cast(half8, q[2]);
    w.li = __builtin_bit_cast(half8, q[3]);
    return w;
}

// LDS positions and twiddle rows of matrix-core pass I as functions of the
// wave, the lane, the group g of 16 butterflies and the point t read or the
// output i written: the expressions of pass16_mfma.  Where every lane of every
// wave sees the same differences from its (g, t) = (0, 0) position as lane 0
// of wave 0 (checked exhaustively at compile time: LINEAR), the pass computes
// one position per lane and adds those differences as compile-time offsets,
// so each LDS access uses the instruction's offset field instead of an address
// register of its own.
template <class G, int I> struct Mfma16Pos {
    static constexpr int Ns = G::r0 * (1 << (4 * I));
    static constexpr int rd(int wv, int lane, int g, int t) {
        const int n = lane & 15, kb = lane >> 4;
        const int b = wv * 64 + g * 16 + n;
        const int c = b >> (G::logL - 4), bb = b & (G::L16 - 1);
        return G::idx(0, c, bb + (4 * kb + t) * G::L16);
    }
    static constexpr int twk(int wv, int lane, int g) {
        const int b = wv * 64 + g * 16 + (lane & 15);
        return (b & (G::L16 - 1)) & (Ns - 1);
    }
    static constexpr int wr(int wv, int lane, int g, int i) {
        const int n = lane & 15, kb = lane >> 4;
        const int b = wv * 64 + g * 16 + n;
        const int c = b >> (G::logL - 4), bb = b & (G::L16 - 1);
        const int k = bb & (Ns - 1);
        return G::idx(0, c, ((bb - k) << 4) + k + (4 * kb + i) * Ns);
    }
    static constexpr bool linear() {
        for (int wv = 0; wv < G::TPP / 64; ++wv)
            for (int lane = 0; lane < 64; ++lane)
                for (int g = 0; g < 4; ++g) {
                    if (twk(wv, lane, g) - twk(wv, lane, 0) != twk(0, 0, g) - twk(0, 0, 0)) return false;
                    for (int t = 0; t < 4; ++t)
                        if (rd(wv, lane, g, t) - rd(wv, lane, 0, 0) != rd(0, 0, g, t) - rd(0, 0, 0, 0) ||
                            wr(wv, lane, g, t) - wr(wv, lane, 0, 0) != wr(0, 0, g, t) - wr(0, 0, 0, 0))
                            return false;
                }
        return true;
    }
    static constexpr bool LINEAR = linear();
    struct Tab {
        int rd[4][4], wr[4][4], tw[4];
    };
    static constexpr Tab tab() {
        Tab r{};
        for (int g = 0; g < 4; ++g) {
            r.tw[g] = twk(0, 0, g) - twk(0, 0, 0);
            for (int t = 0; t < 4; ++t) {
                r.rd[g][t] = rd(0, 0, g, t) - rd(0, 0, 0, 0);
                r.wr[g][t] = wr(0, 0, g, t) - wr(0, 0, 0, 0);
            }
        }
        return r;
    }
};

// Radix-16 pass I as in pass16 (same inputs, twiddles and output positions),
// on the matrix cores.  Every pass, the last included, writes its outputs to
// LDS; the last one's land in natural order.  PREC 1: MFMA_FP16, 2: FP16X2.
template <class G, int I, int PREC, bool WAVE = false>
__device__ __forceinline__ void pass16_mfma(float *sre, float *sim, int pol, int lt, const float2 *tw,
                                            const MfmaW &W) {
    constexpr int Ns = G::r0 * (1 << (4 * I));
    constexpr int GR = 4;  // groups of 16 butterflies per wave
    const int lane = lt & 63, wv = lt >> 6;
    const int n = lane & 15, kb = lane >> 4;
    typedef Mfma16Pos<G, I> Pos;
    constexpr typename Pos::Tab D = Pos::tab();
    // this lane's (g, t) = (0, 0) positions (used where Pos::LINEAR)
    const int b0 = wv * 64 + n;
    const int c0 = b0 >> (G::logL - 4), bb0 = b0 & (G::L16 - 1), k0 = bb0 & (Ns - 1);
    const int rd0 = G::idx(pol, c0, bb0 + 4 * kb * G::L16);
    const int wr0 = G::idx(pol, c0, ((bb0 - k0) << 4) + k0 + 4 * kb * Ns);
    float2 x[GR][4];
#pragma unroll
    for (int g = 0; g < GR; ++g) {
        const int b = wv * 64 + g * 16 + n;
        const int c = b >> (G::logL - 4), bb = b & (G::L16 - 1);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int a = Pos::LINEAR ? rd0 + D.rd[g][t] : G::idx(pol, c, bb + (4 * kb + t) * G::L16);
            x[g][t] = make_float2(sre[a], sim[a]);
        }
        if (Ns > 1) {
            const int k = Pos::LINEAR ? k0 + D.tw[g] : bb & (Ns - 1);
            const float2 *tk = tw + G::tw_off(I) + k * 15;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int r = 4 * kb + t;
                if (r > 0) x[g][t] = cmul(x[g][t], tk[r - 1]);
            }
        }
    }
    pass_sync<WAVE>();
#pragma unroll
    for (int g = 0; g < GR; ++g) {
        // per-butterfly power-of-two scale (lanes n, n+16, n+32, n+48)
        float mx = fmaxf(fmaxf(fabsf(x[g][0].x), fabsf(x[g][0].y)), fabsf(x[g][1].x));
        mx = fmaxf(fmaxf(mx, fabsf(x[g][1].y)), fabsf(x[g][2].x));
        mx = fmaxf(fmaxf(mx, fabsf(x[g][2].y)), fabsf(x[g][3].x));
        mx = fmaxf(mx, fabsf(x[g][3].y));
        // lanes l, l^16, l^32, l^48: the swaps exchange between rows of 16
        // lanes in registers (each lane ends with its partner's value in one
        // of the two results and its own in the other)
        {
            auto r16 = __builtin_amdgcn_permlane16_swap(__float_as_uint(mx), __float_as_uint(mx), false, false);
            mx = fmaxf(mx, fmaxf(__uint_as_float(r16[0]), __uint_as_float(r16[1])));
            auto r32 = __builtin_amdgcn_permlane32_swap(__float_as_uint(mx), __float_as_uint(mx), false, false);
            mx = fmaxf(mx, fmaxf(__uint_as_float(r32[0]), __uint_as_float(r32[1])));
        }
        const int sc = 15 - __builtin_amdgcn_frexp_expf(mx);
        // (re, im) of a point are adjacent operand halves: one packed
        // round-to-nearest conversion gives both hi parts, the lo parts are
        // the exact FP32 remainders, packed the same way
        uint4 uh, ul;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const float2v xs = {__builtin_amdgcn_ldexpf(x[g][t].x, sc), __builtin_amdgcn_ldexpf(x[g][t].y, sc)};
            const half2v h = __builtin_convertvector(xs, half2v);
            const unsigned hu = __builtin_bit_cast(unsigned, h);
            unsigned lu = 0;
            if constexpr (PREC == 2) {
                // x - hi, exact (hi is x rounded to FP16), each in one
                // mixed-precision FMA that widens its FP16 operand itself
                // (instead of a conversion and a subtraction: same bits)
                float rx, ry;
                asm("v_fma_mix_f32 %0, %1, -1.0, %2 op_sel_hi:[1,0,0]" : "=v"(rx) : "v"(hu), "v"(xs.x));
                asm("v_fma_mix_f32 %0, %1, -1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(ry) : "v"(hu), "v"(xs.y));
                const float2v r = {rx, ry};
                lu = __builtin_bit_cast(unsigned, __builtin_convertvector(r, half2v));
            }
            if (t == 0) { uh.x = hu; ul.x = lu; }
            else if (t == 1) { uh.y = hu; ul.y = lu; }
            else if (t == 2) { uh.z = hu; ul.z = lu; }
            else { uh.w = hu; ul.w = lu; }
        }
        const half8 bh = __builtin_bit_cast(half8, uh);
        const half8 bl = __builtin_bit_cast(half8, ul);
        floatx4 yr = {0.f, 0.f, 0.f, 0.f}, yi = {0.f, 0.f, 0.f, 0.f};
        if constexpr (PREC == 2) {
            // small terms first: Wlo*hi, Whi*lo, then Whi*hi
            yr = __builtin_amdgcn_mfma_f32_16x16x32_f16(W.lr, bh, yr, 0, 0, 0);
            yi = __builtin_amdgcn_mfma_f32_16x16x32_f16(W.li, bh, yi, 0, 0, 0);
            yr = __builtin_amdgcn_mfma_f32_16x16x32_f16(W.hr, bl, yr, 0, 0, 0);
            yi = __builtin_amdgcn_mfma_f32_16x16x32_f16(W.hi, bl, yi, 0, 0, 0);
        }
        yr = __builtin_amdgcn_mfma_f32_16x16x32_f16(W.hr, bh, yr, 0, 0, 0);
        yi = __builtin_amdgcn_mfma_f32_16x16x32_f16(W.hi, bh, yi, 0, 0, 0);
        const int b = wv * 64 + g * 16 + n;
        const int c = b >> (G::logL - 4), bb = b & (G::L16 - 1);
        const int k = bb & (Ns - 1);
        const int base = ((bb - k) << 4) + k;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int a = Pos::LINEAR ? wr0 + D.wr[g][i] : G::idx(pol, c, base + (4 * kb + i) * Ns);
            sre[a] = __builtin_amdgcn_ldexpf(yr[i], -sc);
            sim[a] = __builtin_amdgcn_ldexpf(yi[i], -sc);
        }
    }
    pass_sync<WAVE>();
}

template <class G, int I, int PREC, bool WAVE = false>
__device__ __forceinline__ void passes16_mfma(float *sre, float *sim, int pol, int lt, const float2 *tw,
                                              const MfmaW &W) {
    pass16_mfma<G, I, PREC, WAVE>(sre, sim, pol, lt, tw, W);
    if constexpr (I + 1 < G::n16) passes16_mfma<G, I + 1, PREC, WAVE>(sre, sim, pol, lt, tw, W);
}

// The batched FFT of fft_plane with its radix-16 passes on the matrix cores;
// the result is left in LDS in natural order (column c, bin k at idx(pol, c,
// k)).  Without WAVE it ends with a workgroup barrier.  With WAVE (each column
// within the lanes of one wave: a wave's 64 butterflies of every pass, the 4
// groups of 16 that it gives the matrix cores, are whole columns) the passes
// synchronise per wave only, and on return only the calling wave's columns
// are known complete.
template <class G, int PREC, bool WAVE = false>
__device__ __forceinline__ void fft_plane_mfma(float *sre, float *sim, int pol, int lt, const float2 *tw,
                                               const MfmaW &W) {
    static_assert(G::TPP % 64 == 0, "whole waves per polarisation");
    static_assert(!WAVE || G::WAVE_COLS, "wave-local passes need columns within one wave");
    if constexpr (G::r0 > 1) pass_small<G, G::r0, WAVE>(sre, sim, pol, lt);
    passes16_mfma<G, 0, PREC, WAVE>(sre, sim, pol, lt, tw, W);
}

// Precision dispatch: on return thread lt holds X_c[bb + r*L/16] in v (as
// fft_plane), and with IN_LDS the whole transform is also in LDS in natural
// order (matrix-core passes only).  WAVE: the FP32 passes synchronise per
// wave where the geometry allows it (see fft_plane).
// PREC: 0 FP32, 1 FP16 matrix cores, 2 split-FP16 matrix cores, 3 FP64 (row
// pass only; vector ALUs, fft_plane in double).
template <int PREC> struct FftPrec { static constexpr bool IN_LDS = PREC == 1 || PREC == 2; };
template <class G, int PREC> struct FftWave {
    static constexpr bool value = (PREC == 0 || PREC == 3) && G::WAVE_COLS;
};

// MFMA_WAVE (callers that afterwards touch only their own positions until a
// workgroup barrier, as the column passes do): the matrix-core passes also
// synchronise per wave where the geometry allows it.
template <class G, int PREC, bool MFMA_WAVE = false>
__device__ __forceinline__ void fft_plane_p(float *sre, float *sim, int pol, int lt, const float2 *tw,
                                            const MfmaW &W, float2 (&v)[16], bool want_regs) {
    if constexpr (PREC == 0) {
        fft_plane<G, FftWave<G, PREC>::value>(sre, sim, pol, lt, tw, v);
    } else {
        fft_plane_mfma<G, PREC, MFMA_WAVE && G::WAVE_COLS>(sre, sim, pol, lt, tw, W);
        if (want_regs) {
            const int c = lt >> (G::logL - 4), bb = lt & (G::L16 - 1);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int a = G::idx(pol, c, bb + r * G::L16);
                v[r] = make_float2(sre[a], sim[a]);
            }
        }
    }
}

// ---------------------------------------------------------------- unpack --

// One time sample: NPOL complex int8 values, two's complement, exact in float.
template <int NPOL> struct Sample;
// word4: four consecutive time samples, loaded with one 16-byte (dual) or
// 8-byte (single polarisation) access.
template <> struct Sample<2> {
    typedef uint32_t word;
    typedef uint4 word4;
    __device__ __forceinline__ static void unpack(word w, float2 (&x)[2]) {
        x[0] = make_float2((float)(int8_t)(w & 0xff), (float)(int8_t)((w >> 8) & 0xff));
        x[1] = make_float2((float)(int8_t)((w >> 16) & 0xff), (float)(int8_t)(w >> 24));
    }
    __device__ __forceinline__ static word part(const word4 &v, int e) {
        return e == 0 ? v.x : e == 1 ? v.y : e == 2 ? v.z : v.w;
    }
};
template <> struct Sample<1> {
    typedef uint16_t word;
    typedef uint2 word4;
    __device__ __forceinline__ static void unpack(word w, float2 (&x)[1]) {
        x[0] = make_float2((float)(int8_t)(w & 0xff), (float)(int8_t)(w >> 8));
    }
    __device__ __forceinline__ static word part(const word4 &v, int e) {
        const uint32_t d = e < 2 ? v.x : v.y;
        return (word)((e & 1) ? (d >> 16) : (d & 0xffff));
    }
};

__device__ __forceinline__ float part4(const float4 &v, int e) {
    return e == 0 ? v.x : e == 1 ? v.y : e == 2 ? v.z : v.w;
}

// Base address of frame f (block if f >= fs, else tap history).
template <int NPOL>
__device__ __forceinline__ const typename Sample<NPOL>::word *frame_ptr(const Frames &fr, long long f,
                                                                        long long N) {
    typedef typename Sample<NPOL>::word W;
    return f >= fr.fs ? reinterpret_cast<const W *>(fr.blk) + (f - fr.fs) * N
                      : reinterpret_cast<const W *>(fr.hist) + (f - fr.hf0) * N;
}

// y += h * x for one tap; taps are applied in order p = 0..P-1 starting from
// y = 0, so the first one is y = h*x exactly rounded.
template <int NPOL>
__device__ __forceinline__ void tap_fma(float2 (&y)[NPOL], float h, typename Sample<NPOL>::word w) {
    float2 x[NPOL];
    Sample<NPOL>::unpack(w, x);
#pragma unroll
    for (int pol = 0; pol < NPOL; ++pol) {
        y[pol].x = fmaf(h, x[pol].x, y[pol].x);
        y[pol].y = fmaf(h, x[pol].y, y[pol].y);
    }
}

// -------------------------------------------------------------- chunks ----

__device__ __forceinline__ void chunk_range(const Chunks &ch, long long gid, long long &js,
                                            long long &je) {
    const long long d = gid / ch.C, c = gid - d * ch.C;
    js = d * ch.n_int + c * ch.G;
    je = min(js + (long long)ch.G, (d + 1) * ch.n_int);
    js = max(js, ch.j_lo);
    je = min(je, ch.j_hi);
}

// ------------------------------------------------------------- products ---

// |X|^2, |Y|^2, Re X Y*, Im X Y* (Section 4 of the paper).
__device__ __forceinline__ void prod4(float (&acc)[4], float2 X, float2 Y) {
    acc[0] += X.x * X.x + X.y * X.y;
    acc[1] += Y.x * Y.x + Y.y * Y.y;
    acc[2] += X.x * Y.x + X.y * Y.y;
    acc[3] += X.y * Y.x - X.x * Y.y;
}

// The same from double-precision spectra, each product rounded once to FP32
// before it is accumulated.
__device__ __forceinline__ void prod4(float (&acc)[4], double2 X, double2 Y) {
    acc[0] += (float)(X.x * X.x + X.y * X.y);
    acc[1] += (float)(Y.x * Y.x + Y.y * Y.y);
    acc[2] += (float)(X.x * Y.x + X.y * Y.y);
    acc[3] += (float)(X.y * Y.x - X.x * Y.y);
}

}  // namespace pfbs
