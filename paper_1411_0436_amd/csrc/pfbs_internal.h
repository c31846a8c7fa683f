// Internal declarations shared by the host plan code and the HIP kernels.
// Not part of the public ABI (include/pfbspec.h).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pfbs {

constexpr int kTilePoints = 4096;    // T * L: complex points per polarisation per workgroup step
constexpr int kMaxSinglePass = 4096; // largest N done by one kernel (T = 1)

// Points per polarisation per workgroup step of the row pass: whole rows, at
// least 1024 (whole waves per polarisation; 2048 measured slower).
constexpr int back_tile_points(long long n1) { return n1 < 1024 ? 1024 : (int)n1; }

// Arithmetic of the row pass of the two-pass FFT for an FP32 plan: from 2^18
// channels it runs in FP64 on the vector ALUs (internal precision code 3;
// these ALUs issue FP64 at their unpacked FP32 rate).  A strong tone's energy
// sits in one intermediate row, and an FP32 row FFT spreads the rounding of
// that row over all of its channels: on the largest mode (N = 2^19, 64
// spectra per dump) FP32 rows miss 1e-5 per channel in some dumps (1.2e-5),
// with 16 spectra per dump by more (1.7e-5).
constexpr int kRowF64 = 3;
constexpr int fp32_row_precision(long long N) { return N >= (1LL << 18) ? kRowF64 : 0; }

// Column length of the two-pass FFT when the description leaves it open
// (measured fastest): 128 up to 2^15 channels (whole 128-byte int8 rows per
// column tile), 256 above.
constexpr long long default_split(long long N) { return N <= (1LL << 15) ? 128 : 256; }

// Splits that keep a precision's accuracy (the autotuner's candidates): rows
// no longer than the default split's, since the rounding of a strong tone's
// row grows with the row FFT's length; any split where the rows run in FP64
// (FP32 plans from 2^18 channels).  precision: a pfbs_precision value.
constexpr bool split_keeps_accuracy(long long N, int precision, long long n2) {
    return n2 >= default_split(N) || (precision == 0 && fp32_row_precision(N) == kRowF64);
}

// LDS words allocated per column of an L-point sub-FFT plane: one pad word
// per 16 elements and one more per column (the larger of the two layouts the
// kernels use; pads of 0, 3 and 9 words per column measured no better).
constexpr int lds_pitch(int L) { return L + L / 16 + 1; }

// Runtime view of the batched sub-FFT geometry (the kernels take L as a
// template parameter; the host keeps these facts and the twiddle table).
struct Geo {
    int L;
    int T;                // sequences per workgroup step (tile points / L)
    const float2 *tw;     // radix-16 pass twiddles, passes concatenated
    const double2 *tw64;  // the same in FP64 (row pass in FP64 only, else null)
    const uint4 *mw;      // matrix-core DFT-16 operands, [64 lanes][4] (matrix-core plans)
};

// Spectrum-chunk enumeration.  Dump d covers global spectra
// [d*n_int, (d+1)*n_int); each dump is cut into C = ceil(n_int/G) chunks of
// G spectra; global chunk id = d*C + c.  A launch covers chunk ids
// [gid0, gid0 + n_chunks) and spectra [j_lo, j_hi).
struct Chunks {
    long long n_int;
    long long C;
    int G;
    long long j_lo, j_hi;     // spectra of the whole block
    long long gid_lo;         // first chunk id of the block (partial index base)
    long long gid0;           // first chunk id of this launch
};

// Frame addressing of the stream: frame f lives in the block if f >= fs,
// otherwise in the tap history whose first frame is hf0.
struct Frames {
    const uint8_t *blk;
    const uint8_t *hist;
    long long fs, hf0;
};

struct FrontArgs {
    Frames fr;
    const float *taps;        // h[P][N]
    Geo g;
    long long N, N1, N2;      // N1 == 1: single pass (whole FFT here)
    int P;
    int ntiles;               // column tiles along n1 (four-step pass A)
    Chunks ch;
    // pass A: spectra [sa0, sa1) in runs of ga per workgroup
    long long sa0, sa1;
    int ga;
    int znt;                  // 1: streaming (non-temporal) stores of Z
    int pair;                 // 1: two spectra per workgroup step (runs of 2*ga)
    int pt;                   // compile-time tap count of the kernel (4 or 8), 0 = loop over P
    float2 *Z;                // [spectra of launch][pol][N2][N1]
    long long jz0;            // spectrum index of Z[0]
    const float2 *tw4;        // [n1][k2] = W_N^(n1*k2), N entries
    // single-pass output
    float *part;              // [chunks of block][n_prod][N]
};

struct BackArgs {
    const float2 *Z;
    int znt;                  // 1: streaming (non-temporal) loads of Z
    long long jz0;
    Geo g;                    // L = N1
    long long N, N1, N2;
    int ntiles;               // row tiles along k2
    Chunks ch;
    float *part;              // [chunks of block][n_prod][N], index u = k2*N1 + k1
};

struct ReduceArgs {
    const float *part;
    const float *carried_in;  // [n_prod][N], internal order u: sum so far of the dump begun earlier
    float *carried_out;       // [n_prod][N]: sum of the dump left incomplete by this block
    float *out;               // [dumps][n_prod][N], natural order k
    long long N, N1, N2;      // u = k2*N1 + k1  <->  k = k2 + N2*k1 (N2 == 1: identity)
    int n_prod;
    long long n_int, C;
    int G;
    long long j_lo, j_hi, gid_lo, gid_hi, d_lo;
    int flush;                // 1: out[q][k] = carried_in (or 0 if !have_carried)
    int have_carried;
};

// ---- batched launches: one dispatcher kernel per phase serves every
// sub-band of a batch; each workgroup finds its entry by its block id.
constexpr int kMaxBatch = 64;

struct BatchFrontEntry {
    int kind;        // 0 = single pass, 1 = column pass, 2 = two-spectra column pass
    int pfb;
    int L;
    int pt;          // compile-time tap count of the body (4, 8; 0 = from the arguments)
    int wg0, wgn;    // the entry's workgroups are [wg0, wg0 + wgn) of the launch
    int items;       // the body's block count (kinds 0 and 1: two per workgroup)
    FrontArgs a;
};

struct BatchBackEntry {
    int L;
    int prec;        // row arithmetic: 0 FP32, 2 split FP16 on the matrix cores, 3 FP64
    int wg0, wgn;
    int items;       // the body's block count (row phase with single passes: two per workgroup)
    BackArgs a;
};

struct BatchTailEntry {
    int kind;        // 0 = dump reduction, 1 = tap history
    int wg0, wgn;
    int gx, gy;      // reduction grid x, y (z = products)
    ReduceArgs r;
    uint8_t *hdst;   // history
    Frames fr;
    long long F, frame_vec;
    int H;
};

// Kernels of the batched launches (k_batch.hip, k_aux.hip): the front phase,
// the row phase at tile size tp (1024, 2048 or 4096 points), the tail.
const void *batch_front_fn(int npol, bool with_single);
const void *batch_back_fn(int npol, int tp);
const void *batch_rows_single_fn(int npol);   // 2048-point row tiles + single passes
// Compile-time tap count of the pre-filter kernels for P taps (0: taken from
// the arguments at run time; also 0 without the filter or when not unrolled).
constexpr int tap_variant(bool pfb, int P, bool unroll) { return unroll && pfb && (P == 4 || P == 8) ? P : 0; }
const void *batch_tail_fn();

}  // namespace pfbs

#include "../../include/pfbspec.h"

namespace pfbs {

// Kernel timing without extra stream packets: while `start` is set, the next
// library launch on this thread records its start and stop timestamps into
// the two events through the dispatch itself (hipExtLaunchKernel).
struct LaunchEvents {
    hipEvent_t start, stop;
};
extern thread_local LaunchEvents g_launch_events;

#define PFBS_LAUNCH(kernel, grid, block, lds, stream, ...)                                             \
    do {                                                                                               \
        if (::pfbs::g_launch_events.start)                                                             \
            hipExtLaunchKernelGGL(kernel, grid, block, lds, stream, ::pfbs::g_launch_events.start,     \
                                  ::pfbs::g_launch_events.stop, 0, __VA_ARGS__);                       \
        else                                                                                           \
            hipLaunchKernelGGL(kernel, grid, block, lds, stream, __VA_ARGS__);                         \
    } while (0)

// Set the calling thread's pfbs_last_error text and return st (plan.cpp).
pfbs_status record_error(pfbs_status st, const char *msg);
// The checks of pfbs_plan_create_ex on a description, leaving the calling
// thread's pfbs_last_error text as it was (plan.cpp).
pfbs_status validate_desc_quiet(const pfbs_plan_desc *d);

// ---- autotune cache (autotune.cpp) ----
// Fill *out from the newest cache line matching desc's shape on the current
// device (speed-only fields); with measure_if_missing, run the autotuner when
// there is none.  Leaves *out = *desc when nothing applies.
pfbs_status tune_lookup(const pfbs_plan_desc *desc, bool measure_if_missing, pfbs_plan_desc *out);
hipError_t launch_synth(uint32_t *words, long long n_words, uint32_t seed, hipStream_t s);

// ---- launchers (kernels.hip) ----
hipError_t launch_tables_taps(float *h, long long N, int P, int window, const double *d_custom,
                              hipStream_t s);
hipError_t launch_tables_tw16(float2 *tw, int L, hipStream_t s);
hipError_t launch_tables_tw16_f64(double2 *tw, int L, hipStream_t s);
hipError_t launch_tables_mfma(uint4 *mw, hipStream_t s);   // 64 lanes x 4 uint4
hipError_t launch_tables_tw4(float2 *tw4, long long N1, long long N2, hipStream_t s);
// prec: 0 = FP32, 1 = matrix cores with an FP16 DFT matrix, 2 = hi + lo matrix
hipError_t launch_front(const FrontArgs &a, int npol, bool pfb, bool single, int prec, int n_items,
                        hipStream_t s);
hipError_t launch_back(const BackArgs &a, int npol, int prec, int n_chunks, hipStream_t s);
// the row pass by arithmetic (k_rows_f32.hip: 0 and kRowF64; k_rows_mfma.hip: 1 and 2)
hipError_t launch_back_vector(const BackArgs &a, int npol, int prec, int n_chunks, hipStream_t s);
hipError_t launch_back_mfma(const BackArgs &a, int npol, int prec, int n_chunks, hipStream_t s);
hipError_t init_back_vector(int lds_limit);
hipError_t init_back_mfma(int lds_limit);
hipError_t launch_reduce(const ReduceArgs &a, int n_dumps, hipStream_t s);
// In place on n_dumps rows of [n_prod][N]: products -> Stokes, and/or the
// shifted channel order.
hipError_t launch_dump_format(float *out, long long n_dumps, long long N, int n_prod, int stokes, int shift,
                              hipStream_t s);
hipError_t launch_history(uint8_t *dst, const Frames &fr, long long F, int H, long long frame_bytes,
                          hipStream_t s);
// launch_reduce and launch_history as one launch
hipError_t launch_reduce_history(const ReduceArgs &a, int n_dumps, uint8_t *dst, const Frames &fr, long long F,
                                 int H, long long frame_bytes, hipStream_t s);
hipError_t launch_debug_pfb(float *y, const Frames &fr, const float *taps, long long N, int P,
                            int npol, bool pfb, long long j_lo, long long j_hi, hipStream_t s);
hipError_t kernels_init();   // raise LDS limits once per process/device
bool init_fourstep_pair(int lds_limit);  // LDS limit of the two-spectra column kernels; false if refused
bool init_batch(int lds_limit);          // LDS limit of the batched phase kernels; false if refused
size_t front_lds_bytes(const Geo &g, int npol);
size_t back_lds_bytes(const Geo &g, int npol, int prec);

}  // namespace pfbs
