// Host side of the spectrometer library: plan objects, argument validation,
// block / spectrum / dump bookkeeping and the launch sequence per block.
//
// The split follows the paper's high-level algorithm (Section 4): plan
// creation is its initialisation (filter coefficients to the device, FFT
// planned for the parallel transforms), pfbs_execute is one turn of its loop
// (pre-filter, parallel FFTs, accumulation) on a block that is already in
// device memory.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/pfbspec.h"
#include "pfbs_internal.h"

using namespace pfbs;

namespace {

thread_local std::string g_err;

pfbs_status fail(pfbs_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

}  // namespace

namespace pfbs {
thread_local LaunchEvents g_launch_events = {nullptr, nullptr};

pfbs_status record_error(pfbs_status st, const char *msg) {
    g_err = msg;
    return st;
}
}  // namespace pfbs

namespace {

constexpr uint32_t kMagic = 0x50464253u;  // "PFBS"
constexpr uint32_t kDead = 0xdeadbeefu;

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }
int ilog2(int64_t v) {
    int r = 0;
    while ((int64_t(1) << r) < v) ++r;
    return r;
}

// tp: complex points per polarisation per workgroup step of the kernel.
Geo make_geo(int L, int tp = kTilePoints) {
    Geo g{};
    g.L = L;
    g.T = tp / L;
    g.tw = nullptr;
    return g;
}

// Entries of the radix-16 pass twiddle table for length L = r0 * 16^n16:
// sum over passes of Ns*15 with Ns = r0, 16 r0, ...
int64_t tw16_count(const Geo &g) {
    const int logL = ilog2(g.L);
    int64_t n = 0, Ns = int64_t(1) << (logL % 4);
    for (int i = 0; i < logL / 4; ++i) {
        n += Ns * 15;
        Ns *= 16;
    }
    return n;
}

std::mutex g_init_mu;
bool g_init_done[64];

// Scratch memory of pfbs_execute_noalloc: a file-scope device array (each
// device the library runs on holds its own copy until the process ends).  In
// host code its name is not a device address; the address comes from
// hipGetSymbolAddress, taken once per device at its first plan creation.
constexpr size_t kNoAllocScratch = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratch];
void *g_scratch_ptr[64];
// Column pass on two spectra per workgroup step: its LDS (twice the one-spectrum
// kernel's, up to 140 KB) is available on the device.
bool g_pair_ok[64];
bool g_batch_ok[64];
constexpr int kPairLds = 160 * 1024;

}  // namespace

struct pfbs_plan {
    uint32_t magic;
    // description
    int64_t N;
    int32_t P;
    int32_t window, mode, npol, precision, device;
    int prec_front, prec_back;  // kernel arithmetic of the single/column pass and of the row pass
    int64_t n_int;
    int32_t nprod;
    bool pfb;
    // geometry
    bool fourstep;
    int64_t N1, N2;
    Geo gA, gB;
    int ntilesA, ntilesB;
    int G;
    int64_t C;
    int64_t group_spectra;
    int ga_force;        // column-pass spectra per workgroup (0 = automatic)
    int out_stokes, out_shift;  // dump form: Stokes parameters, shifted channel order
    int znt;             // streaming stores/loads of the four-step intermediate
    int tap_unroll;      // pre-filter tap loop: 1 unrolled at compile time, 2 run-time loop
    bool pair;           // FP32 pre-filter column pass on two spectra per workgroup step
    // device state
    float *taps;
    float2 *twA, *twB, *tw4;
    double2 *twB64;      // row-pass twiddles in FP64 (FP64 row pass only)
    uint4 *mw;           // matrix-core DFT-16 operands (plans using the matrix cores)
    uint8_t *hist[2];
    int hcur;
    int64_t frame_bytes;
    float2 *Z;
    size_t Zcap;      // float2 elements
    float *part;
    size_t partcap;   // floats
    float *carried[2];   // ping-pong: read the current one, write the other
    int ccur;
    int64_t device_bytes;
    // stream counters
    int64_t frames_seen, spectra_done, dumps_done;
    bool poisoned;
    // host-side fault injection (PFBS_FAULT, read at plan creation): the
    // n-th device allocation / kernel launch of this plan reports a failure
    // instead of being made (0 = off)
    int64_t fault_alloc, fault_launch;
    // optional kernel timing: (kind, start, stop) per launch since the last read
    uint32_t timing;     // bit k: time the launches of kernel kind k
    std::vector<hipEvent_t> ev_pool;
    struct Rec { int kind; int i0; };
    std::vector<Rec> recs;
    size_t ev_used;
};

struct pfbs_batch {
    uint32_t magic;
    std::vector<pfbs_plan *> plans;
    int npol;
    int tpb;        // row-phase tile points per polarisation (1024, 2048 or 4096)
    bool rows_single;  // single passes run in the row phase (2048-point row tiles)
    int launches;   // kernel launches made by the last execute
    // entry tables, a ring of kTabRing buffers: buffer k is filled on the
    // host, copied to the device on the batch's copy stream while the
    // caller's stream still runs earlier blocks, and read by the kernels of
    // the execute that filled it.  The host waits only for the upload of
    // kTabRing executes back, so it can stay that many blocks ahead.
    struct Tables {
        BatchFrontEntry front[kMaxBatch];
        BatchBackEntry back[kMaxBatch];
        BatchTailEntry tail[2 * kMaxBatch];
    };
    static constexpr int kTabRing = 4;
    Tables *d_tab[kTabRing];
    Tables *h_tab[kTabRing];
    hipEvent_t copied[kTabRing];   // upload of buffer k done (its host copy is free)
    hipEvent_t done[kTabRing];     // kernels that read device buffer k done
    int stage;
    hipStream_t cstream;    // table copies
    // HIP graphs of the three launches (one per table buffer) with upper-bound
    // grids, captured on a stream of their own on first use for one set of
    // block sizes, replayed on the caller's stream
    hipStream_t gstream;
    hipGraph_t graph[kTabRing];
    hipGraphExec_t gexec[kTabRing];
    std::vector<int64_t> gsizes[kTabRing];
};

namespace {

pfbs_status hip_fail(pfbs_plan *p, hipError_t e, const char *what) {
    if (p) p->poisoned = true;
    return fail(e == hipErrorOutOfMemory ? PFBS_ERR_NOMEM : PFBS_ERR_DEVICE, "%s: %s", what,
                hipGetErrorString(e));
}

#define PFBS_HIP(p, call)                                   \
    do {                                                    \
        hipError_t _e = (call);                             \
        if (_e != hipSuccess) return hip_fail((p), _e, #call); \
    } while (0)

// Column length N2 (pass A) and row length N1 = N/N2 (pass B) of the
// two-pass FFT: both must have kernels built for them and tile evenly.
int back_tile(int64_t n1) { return back_tile_points(n1); }  // row-pass points per pol

bool split_ok(int64_t N, int64_t n2) {
    if (!is_pow2(n2) || n2 < 64 || n2 > 512) return false;
    const int64_t n1 = N / n2;
    if (n1 < 32 || n1 > kMaxSinglePass) return false;
    return n1 % (kTilePoints / n2) == 0 && n2 % (back_tile(n1) / n1) == 0;
}

pfbs_status validate_desc(const pfbs_plan_desc *d) {
    if (!d) return fail(PFBS_ERR_INVALID, "desc is NULL");
    if (!is_pow2(d->N) || d->N < 16 || d->N > (int64_t(1) << 20))
        return fail(PFBS_ERR_INVALID, "N=%lld must be a power of two in [16, 2^20]", (long long)d->N);
    if (d->P < 1 || d->P > 16) return fail(PFBS_ERR_INVALID, "P=%d must be in [1, 16]", d->P);
    if (d->mode != PFBS_MODE_PFB && d->mode != PFBS_MODE_DIRECT)
        return fail(PFBS_ERR_INVALID, "unknown mode %d", d->mode);
    if (d->mode == PFBS_MODE_DIRECT && d->P != 1)
        return fail(PFBS_ERR_INVALID, "direct mode requires P=1 (got %d)", d->P);
    if (d->window != PFBS_WINDOW_HANN_SINC && d->window != PFBS_WINDOW_RECT &&
        d->window != PFBS_WINDOW_CUSTOM)
        return fail(PFBS_ERR_INVALID, "unknown window %d", d->window);
    if (d->mode == PFBS_MODE_PFB && d->window == PFBS_WINDOW_CUSTOM && !d->custom_taps)
        return fail(PFBS_ERR_INVALID, "custom window needs custom_taps");
    if (d->n_pol != 1 && d->n_pol != 2) return fail(PFBS_ERR_INVALID, "n_pol=%d must be 1 or 2", d->n_pol);
    if (d->n_int < 1) return fail(PFBS_ERR_INVALID, "n_int=%lld must be >= 1", (long long)d->n_int);
    if (d->precision != PFBS_PREC_FP32 && d->precision != PFBS_PREC_MFMA_FP16 &&
        d->precision != PFBS_PREC_MFMA_FP16X2 && d->precision != PFBS_PREC_MIXED)
        return fail(PFBS_ERR_INVALID, "unknown precision %d", d->precision);
    if (d->chunk < 0 || d->chunk > 65536) return fail(PFBS_ERR_INVALID, "chunk=%d out of range", d->chunk);
    if (d->split_n2 != 0) {
        if (d->N <= kMaxSinglePass)
            return fail(PFBS_ERR_INVALID, "split_n2 given but N=%lld is done in one pass", (long long)d->N);
        if (!split_ok(d->N, d->split_n2))
            return fail(PFBS_ERR_INVALID, "split_n2=%lld invalid for N=%lld (column length 64..512, "
                        "row length 32..4096)", (long long)d->split_n2, (long long)d->N);
    }
    if (d->row_tile != 0 && d->N > kMaxSinglePass) {
        const int64_t n2 = d->split_n2 ? d->split_n2 : default_split(d->N), n1 = d->N / n2;
        if (d->row_tile < n1 || n2 % (d->row_tile / n1) != 0)
            return fail(PFBS_ERR_INVALID, "row_tile=%d invalid for rows of %lld points", d->row_tile, (long long)n1);
    }
    if (d->group_bytes < 0) return fail(PFBS_ERR_INVALID, "group_bytes < 0");
    if (d->col_run < 0 || d->col_run > 64) return fail(PFBS_ERR_INVALID, "col_run=%d out of [0, 64]", d->col_run);
    if (d->stream_z != 0 && d->stream_z != 1) return fail(PFBS_ERR_INVALID, "stream_z must be 0 or 1");
    if (d->output != PFBS_OUT_PRODUCTS && d->output != PFBS_OUT_STOKES)
        return fail(PFBS_ERR_INVALID, "unknown output form %d", d->output);
    if (d->output == PFBS_OUT_STOKES && d->n_pol != 2)
        return fail(PFBS_ERR_INVALID, "Stokes output needs two polarisations");
    if (d->fftshift != 0 && d->fftshift != 1) return fail(PFBS_ERR_INVALID, "fftshift must be 0 or 1");
    if (d->tune < 0 || d->tune > 2) return fail(PFBS_ERR_INVALID, "tune must be 0, 1 or 2");
    if (d->tap_unroll < 0 || d->tap_unroll > 2) return fail(PFBS_ERR_INVALID, "tap_unroll must be 0, 1 or 2");
    if (d->col_pair < 0 || d->col_pair > 2) return fail(PFBS_ERR_INVALID, "col_pair must be 0, 1 or 2");
    if (d->row_tile != 0 && d->row_tile != 1024 && d->row_tile != 2048 && d->row_tile != 4096)
        return fail(PFBS_ERR_INVALID, "row_tile=%d: 0, 1024, 2048 or 4096", d->row_tile);
    return PFBS_OK;
}

// Spectra of global chunk gid intersected with [j_lo, j_hi).
void chunk_span(const pfbs_plan *p, int64_t gid, int64_t j_lo, int64_t j_hi, int64_t &js, int64_t &je) {
    const int64_t d = gid / p->C, c = gid - d * p->C;
    js = d * p->n_int + c * p->G;
    je = std::min(js + (int64_t)p->G, (d + 1) * p->n_int);
    js = std::max(js, j_lo);
    je = std::min(je, j_hi);
}

int64_t chunk_of(const pfbs_plan *p, int64_t j) {
    const int64_t d = j / p->n_int;
    return d * p->C + (j - d * p->n_int) / p->G;
}

// Spectra [j_lo, j_hi) completed by a block of F frames.
void block_spectra(const pfbs_plan *p, int64_t F, int64_t &j_lo, int64_t &j_hi) {
    const int64_t need = p->pfb ? p->P : 1;
    j_lo = p->spectra_done;
    j_hi = std::max<int64_t>(0, p->frames_seen + F - need + 1);
    if (j_hi < j_lo) j_hi = j_lo;
}

bool plan_ok(const pfbs_plan *p) { return p && p->magic == kMagic; }

template <typename T>
hipError_t dalloc(pfbs_plan *p, T **ptr, size_t count) {
    *ptr = nullptr;
    if (count == 0) count = 1;
    if (p->fault_alloc > 0 && --p->fault_alloc == 0) return hipErrorOutOfMemory;  // injected
    hipError_t e = hipMalloc((void **)ptr, count * sizeof(T));
    if (e == hipSuccess) p->device_bytes += (int64_t)(count * sizeof(T));
    return e;
}

void free_plan_memory(pfbs_plan *p) {
    void *bufs[] = {p->taps, p->twA, p->twB, p->twB64, p->mw, p->tw4, p->hist[0], p->hist[1],
                    p->Z, p->part, p->carried[0], p->carried[1]};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
}

// Run one launch, bracketed by timing events when the plan measures kernels.
template <typename F>
hipError_t timed(pfbs_plan *p, int kind, hipStream_t s, F &&launch) {
    if (p->fault_launch > 0 && --p->fault_launch == 0) return hipErrorLaunchFailure;  // injected
    if (!((p->timing >> kind) & 1u)) return launch();
    while (p->ev_pool.size() < p->ev_used + 2) {
        hipEvent_t e;
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return r;
        p->ev_pool.push_back(e);
    }
    const int i0 = (int)p->ev_used;
    // the launch records its own start/stop timestamps (no extra packets)
    g_launch_events = {p->ev_pool[i0], p->ev_pool[i0 + 1]};
    hipError_t r = launch();
    g_launch_events = {nullptr, nullptr};
    (void)s;
    if (r != hipSuccess) return r;
    p->ev_used += 2;
    p->recs.push_back({kind, i0});
    return hipSuccess;
}

// PFBS_FAULT = "alloc:<n>" or "launch:<n>" (n >= 1): the plan created while
// it is set fails its n-th device allocation (hipErrorOutOfMemory) or its
// n-th kernel launch (hipErrorLaunchFailure) on the host, without touching
// the device, so that the error, poisoning and reset paths can be exercised.
void parse_fault(pfbs_plan *p) {
    p->fault_alloc = p->fault_launch = 0;
    const char *f = getenv("PFBS_FAULT");
    if (!f) return;
    long long n = 0;
    if (sscanf(f, "alloc:%lld", &n) == 1 && n > 0) p->fault_alloc = n;
    else if (sscanf(f, "launch:%lld", &n) == 1 && n > 0) p->fault_launch = n;
}

pfbs_status ensure_scratch(pfbs_plan *p, size_t z_elems, size_t part_floats) {
    if (z_elems > p->Zcap) {
        if (p->Z) {
            (void)hipFree(p->Z);
            p->device_bytes -= (int64_t)(p->Zcap * sizeof(float2));
            p->Z = nullptr;
            p->Zcap = 0;
        }
        PFBS_HIP(p, dalloc(p, &p->Z, z_elems));
        p->Zcap = z_elems;
    }
    if (part_floats > p->partcap) {
        if (p->part) {
            (void)hipFree(p->part);
            p->device_bytes -= (int64_t)(p->partcap * sizeof(float));
            p->part = nullptr;
            p->partcap = 0;
        }
        PFBS_HIP(p, dalloc(p, &p->part, part_floats));
        p->partcap = part_floats;
    }
    return PFBS_OK;
}

}  // namespace

extern "C" {

const char *pfbs_last_error(void) { return g_err.c_str(); }

#ifndef PFBS_SOURCE_DIGEST
#define PFBS_SOURCE_DIGEST "unknown"
#endif
const char *pfbs_version(void) { return "pfbspec " PFBS_SOURCE_DIGEST; }

pfbs_status pfbs_plan_create_ex(pfbs_plan **out, const pfbs_plan_desc *desc_in) {
    if (!out) return fail(PFBS_ERR_INVALID, "out is NULL");
    *out = nullptr;
    pfbs_status st = validate_desc(desc_in);
    if (st != PFBS_OK) return st;
    pfbs_plan_desc tuned = *desc_in;
    if (desc_in->tune != 0) {
        st = pfbs::tune_lookup(desc_in, desc_in->tune == 2, &tuned);
        if (st != PFBS_OK) return st;
        st = validate_desc(&tuned);
        if (st != PFBS_OK) return st;
    }
    const pfbs_plan_desc *desc = &tuned;

    int dev = desc->device;
    if (dev < 0) {
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetDevice");
    } else {
        hipError_t e = hipSetDevice(dev);
        if (e != hipSuccess) return hip_fail(nullptr, e, "hipSetDevice");
    }
    if (dev < 0 || dev >= 64) return fail(PFBS_ERR_UNSUPPORTED, "device ordinal %d", dev);
    {
        std::lock_guard<std::mutex> lk(g_init_mu);
        if (!g_init_done[dev]) {
            hipError_t e = kernels_init();
            if (e != hipSuccess) return hip_fail(nullptr, e, "kernel attributes");
            void *sp = nullptr;
            e = hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch));
            if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetSymbolAddress(scratch)");
            g_scratch_ptr[dev] = sp;
            g_pair_ok[dev] = init_fourstep_pair(kPairLds);
            g_batch_ok[dev] = init_batch(kPairLds);
            g_init_done[dev] = true;
        }
    }

    pfbs_plan *p = new (std::nothrow) pfbs_plan();
    if (!p) return fail(PFBS_ERR_NOMEM, "host allocation");
    p->magic = kMagic;
    parse_fault(p);
    p->N = desc->N;
    p->pfb = desc->mode == PFBS_MODE_PFB;
    p->P = p->pfb ? desc->P : 1;
    p->window = desc->window;
    p->mode = desc->mode;
    p->npol = desc->n_pol;
    p->precision = desc->precision;
    p->prec_front = desc->precision == PFBS_PREC_MIXED ? PFBS_PREC_FP32 : desc->precision;
    p->prec_back = desc->precision == PFBS_PREC_MIXED ? PFBS_PREC_MFMA_FP16X2 : desc->precision;
    if (p->prec_back == PFBS_PREC_FP32) p->prec_back = fp32_row_precision(desc->N);
    p->device = dev;
    p->n_int = desc->n_int;
    p->nprod = p->npol == 2 ? 4 : 1;
    p->fourstep = p->N > kMaxSinglePass;
    if (p->fourstep) {
        p->N2 = desc->split_n2 ? desc->split_n2 : default_split(p->N);
        p->N1 = p->N / p->N2;
        p->gA = make_geo((int)p->N2);
        p->gB = make_geo((int)p->N1, desc->row_tile ? desc->row_tile : back_tile(p->N1));
        p->ntilesA = (int)(p->N1 / p->gA.T);
        p->ntilesB = (int)(p->N2 / p->gB.T);
    } else {
        p->N1 = 1;
        p->N2 = p->N;
        p->gA = make_geo((int)p->N);
        p->ntilesA = 1;
        p->ntilesB = 0;
    }
    if (desc->chunk > 0) p->G = desc->chunk;
    else p->G = p->fourstep ? 16 : std::max(16, p->gA.T);
    p->C = (p->n_int + p->G - 1) / p->G;
    const int64_t zbytes_per_spec = (int64_t)p->npol * p->N * (int64_t)sizeof(float2);
    const int64_t gb = desc->group_bytes > 0 ? desc->group_bytes : (int64_t(1) << 30);
    p->group_spectra = std::max<int64_t>(p->G, gb / zbytes_per_spec);
    p->frame_bytes = p->N * 2 * p->npol;
    p->ga_force = desc->col_run;
    p->znt = desc->stream_z;
    p->tap_unroll = desc->tap_unroll;
    // Two spectra per column-pass step share each tap-row load: measured
    // faster only where the tap table (P*N floats) overflows the 4 MB L2 of
    // an XCD (N = 2^19: column pass -8%; N <= 2^16: +3 to +6%), and with
    // columns of at most 256 (the 512 kernel spills registers).
    const bool pair_fits = p->fourstep && p->pfb && g_pair_ok[dev] && p->gA.L <= 256 &&
                           2 * front_lds_bytes(p->gA, p->npol) <= (size_t)kPairLds;
    // automatic: FP32 columns where the tap table overflows an XCD's L2 (the
    // matrix-core column FFT spills registers in the 1024-thread workgroup:
    // split-FP16 at N=2^19 1010 against 761 us one spectrum per step)
    p->pair = pair_fits && (desc->col_pair == 1 ||
                            (desc->col_pair == 0 && p->prec_front == PFBS_PREC_FP32 &&
                             (int64_t)p->P * p->N >= (int64_t(1) << 21)));
    // tap loop: unrolled where measured faster (the two-spectra column
    // kernel: N=2^19 column pass 570 -> 539 us; the one-spectrum column
    // kernel at N=2^15 180 against 131 us rolled)
    if (p->tap_unroll == 0) p->tap_unroll = p->pair ? 1 : 2;
    p->out_stokes = desc->output == PFBS_OUT_STOKES;
    p->out_shift = desc->fftshift;

    hipStream_t s = nullptr;
    double *d_custom = nullptr;
    pfbs_status rs = PFBS_OK;
    hipError_t e = hipSuccess;
    do {
        if ((e = dalloc(p, &p->taps, (size_t)p->P * p->N)) != hipSuccess) break;
        if ((e = dalloc(p, &p->twA, (size_t)tw16_count(p->gA))) != hipSuccess) break;
        p->gA.tw = p->twA;
        if (p->prec_front == PFBS_PREC_MFMA_FP16 || p->prec_front == PFBS_PREC_MFMA_FP16X2 ||
            p->prec_back == PFBS_PREC_MFMA_FP16 || p->prec_back == PFBS_PREC_MFMA_FP16X2) {
            if ((e = dalloc(p, &p->mw, 64 * 4)) != hipSuccess) break;
            if ((e = launch_tables_mfma(p->mw, s)) != hipSuccess) break;
            p->gA.mw = p->mw;
            p->gB.mw = p->mw;
        }
        if (p->fourstep) {
            if ((e = dalloc(p, &p->twB, (size_t)tw16_count(p->gB))) != hipSuccess) break;
            p->gB.tw = p->twB;
            if (p->prec_back == kRowF64) {
                if ((e = dalloc(p, &p->twB64, (size_t)tw16_count(p->gB))) != hipSuccess) break;
                p->gB.tw64 = p->twB64;
            }
            if ((e = dalloc(p, &p->tw4, (size_t)p->N)) != hipSuccess) break;
        }
        const size_t hbytes = (size_t)(p->P - 1) * p->frame_bytes;
        if (p->P > 1) {
            if ((e = dalloc(p, &p->hist[0], hbytes)) != hipSuccess) break;
            if ((e = dalloc(p, &p->hist[1], hbytes)) != hipSuccess) break;
            if ((e = hipMemsetAsync(p->hist[0], 0, hbytes, s)) != hipSuccess) break;
        }
        if ((e = dalloc(p, &p->carried[0], (size_t)p->nprod * p->N)) != hipSuccess) break;
        if ((e = dalloc(p, &p->carried[1], (size_t)p->nprod * p->N)) != hipSuccess) break;
        int window = p->pfb ? p->window : PFBS_WINDOW_RECT;
        if (window == PFBS_WINDOW_CUSTOM) {
            const size_t n = (size_t)p->P * p->N;
            if ((e = hipMalloc((void **)&d_custom, n * sizeof(double))) != hipSuccess) break;
            if ((e = hipMemcpy(d_custom, desc->custom_taps, n * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess) break;
        }
        if ((e = launch_tables_taps(p->taps, p->N, p->P, window, d_custom, s)) != hipSuccess) break;
        if ((e = launch_tables_tw16(p->twA, p->gA.L, s)) != hipSuccess) break;
        if (p->fourstep) {
            if ((e = launch_tables_tw16(p->twB, p->gB.L, s)) != hipSuccess) break;
            if (p->twB64 && (e = launch_tables_tw16_f64(p->twB64, p->gB.L, s)) != hipSuccess) break;
            if ((e = launch_tables_tw4(p->tw4, p->N1, p->N2, s)) != hipSuccess) break;
        }
        if ((e = hipDeviceSynchronize()) != hipSuccess) break;
    } while (0);
    if (d_custom) (void)hipFree(d_custom);
    if (e != hipSuccess) {
        rs = hip_fail(nullptr, e, "plan creation");
        free_plan_memory(p);
        p->magic = kDead;
        delete p;
        return rs;
    }
    *out = p;
    return PFBS_OK;
}

pfbs_status pfbs_plan_create(pfbs_plan **out, int64_t N, int32_t P, int32_t window, int32_t mode,
                             int32_t n_pol, int64_t n_int) {
    pfbs_plan_desc d;
    memset(&d, 0, sizeof d);
    d.N = N;
    d.P = P;
    d.window = window;
    d.mode = mode;
    d.n_pol = n_pol;
    d.n_int = n_int;
    d.precision = PFBS_PREC_FP32;
    d.device = -1;
    return pfbs_plan_create_ex(out, &d);
}

pfbs_status pfbs_plan_destroy(pfbs_plan *p) {
    if (!p) return PFBS_OK;
    if (!plan_ok(p)) return fail(PFBS_ERR_STATE, "not a live plan");
    (void)hipSetDevice(p->device);
    (void)hipDeviceSynchronize();
    for (hipEvent_t e : p->ev_pool) (void)hipEventDestroy(e);
    free_plan_memory(p);
    p->magic = kDead;
    delete p;
    return PFBS_OK;
}

int64_t pfbs_dumps_in(const pfbs_plan *p, int64_t n) {
    if (!plan_ok(p) || n <= 0 || n % p->N != 0) return -1;
    int64_t j_lo, j_hi;
    block_spectra(p, n / p->N, j_lo, j_hi);
    return j_hi / p->n_int - j_lo / p->n_int;
}

pfbs_status pfbs_plan_get_info(const pfbs_plan *p, pfbs_plan_info *info) {
    if (!plan_ok(p)) return fail(PFBS_ERR_STATE, "not a live plan");
    if (!info) return fail(PFBS_ERR_INVALID, "info is NULL");
    memset(info, 0, sizeof *info);
    info->N = p->N;
    info->P = p->P;
    info->n_pol = p->npol;
    info->n_prod = p->nprod;
    info->mode = p->mode;
    info->precision = p->precision;
    info->chunk = p->G;
    info->n_int = p->n_int;
    info->split_n1 = p->N1;
    info->split_n2 = p->N2;
    info->frames_seen = p->frames_seen;
    info->spectra_done = p->spectra_done;
    info->dumps_done = p->dumps_done;
    info->device_bytes = p->device_bytes;
    info->row_arith = p->fourstep ? p->prec_back : -1;
    info->row_tile = p->fourstep ? p->gB.T * p->gB.L : 0;
    return PFBS_OK;
}

static pfbs_status check_block(const pfbs_plan *p, const void *d_block, int64_t n) {
    if (!plan_ok(p)) return fail(PFBS_ERR_STATE, "not a live plan");
    if (p->poisoned) return fail(PFBS_ERR_STATE, "plan is poisoned by an earlier device error; reset it");
    if (!d_block) return fail(PFBS_ERR_INVALID, "d_block is NULL");
    if (((uintptr_t)d_block & 15) != 0) return fail(PFBS_ERR_INVALID, "d_block must be 16-byte aligned");
    if (n <= 0 || n % p->N != 0)
        return fail(PFBS_ERR_INVALID, "n_time_samples=%lld must be a positive multiple of N=%lld",
                    (long long)n, (long long)p->N);
    return PFBS_OK;
}

}  // extern "C"

namespace {

// One block's work for one plan, computed on the host before any launch.
struct Group {
    FrontArgs fa;
    BackArgs ba;
    int na;   // column-pass items (runs of ga spectra)
    int nc;   // chunks
};

struct Prepared {
    int64_t F = 0, j_lo = 0, j_hi = 0, nd_out = 0;
    bool any = false;
    FrontArgs single{};
    int single_chunks = 0;
    std::vector<Group> groups;
    ReduceArgs ra{};
    int n_dumps = 0;
    bool hist = false;
    Frames fr{};
    bool flip_carried = false;
};

// Validate the block, size the scratch buffers and compute every launch's
// arguments.  Changes no stream state.  one_group: the whole block's
// intermediate in one column pass / row pass pair (batched launches).
// Scratch of one execute: the two-pass intermediate and the chunk partial sums.
struct Scratch {
    float2 *Z;
    size_t Zcap;      // float2 elements
    float *part;
    size_t partcap;   // floats
};

pfbs_status prepare(pfbs_plan *p, const void *d_block, int64_t n, float *d_dumps, int64_t cap,
                    bool one_group, Prepared &w, void *fixed = nullptr, size_t fixed_bytes = 0) {
    pfbs_status st = check_block(p, d_block, n);
    if (st != PFBS_OK) return st;
    w.F = n / p->N;
    block_spectra(p, w.F, w.j_lo, w.j_hi);
    w.nd_out = w.j_hi / p->n_int - w.j_lo / p->n_int;
    if (w.nd_out > 0 && !d_dumps)
        return fail(PFBS_ERR_INVALID, "d_dumps is NULL but %lld dumps complete", (long long)w.nd_out);
    if (cap < w.nd_out)
        return fail(PFBS_ERR_INVALID, "dump_capacity=%lld < %lld dumps completed by this block",
                    (long long)cap, (long long)w.nd_out);
    PFBS_HIP(p, hipSetDevice(p->device));
    w.fr.blk = (const uint8_t *)d_block;
    w.fr.hist = p->hist[p->hcur];
    w.fr.fs = p->frames_seen;
    w.fr.hf0 = p->frames_seen - (p->P - 1);
    w.hist = p->pfb && p->P > 1;
    w.any = w.j_hi > w.j_lo;
    w.groups.clear();
    if (!w.any) return PFBS_OK;
    const int64_t j_lo = w.j_lo, j_hi = w.j_hi;
    const int64_t gid_lo = chunk_of(p, j_lo), gid_hi = chunk_of(p, j_hi - 1);
    const int64_t n_chunks = gid_hi - gid_lo + 1;
    Chunks ch;
    ch.n_int = p->n_int;
    ch.C = p->C;
    ch.G = p->G;
    ch.j_lo = j_lo;
    ch.j_hi = j_hi;
    ch.gid_lo = gid_lo;
    ch.gid0 = gid_lo;
    Scratch sc;
    const size_t part_floats = (size_t)n_chunks * p->nprod * p->N;
    if (fixed) {
        // a caller-independent fixed buffer (no allocation): the partial sums
        // first, the intermediate in the rest; groups are sized to fit it
        const size_t part_bytes = (part_floats * sizeof(float) + 255) & ~(size_t)255;
        const size_t zmin = p->fourstep ? (size_t)p->G * p->npol * p->N * sizeof(float2) : 0;
        if (part_bytes + zmin > fixed_bytes)
            return fail(PFBS_ERR_INVALID,
                        "block needs %zu bytes of scratch (%zu of partial sums, at least %zu of intermediate); "
                        "the allocation-free entry point has %zu: use smaller blocks or a smaller chunk",
                        part_bytes + zmin, part_bytes, zmin, fixed_bytes);
        sc.part = reinterpret_cast<float *>(fixed);
        sc.partcap = part_floats;
        sc.Z = reinterpret_cast<float2 *>(reinterpret_cast<char *>(fixed) + part_bytes);
        sc.Zcap = p->fourstep ? (fixed_bytes - part_bytes) / sizeof(float2) : 0;
    } else {
        size_t zneed = 0;
        if (p->fourstep) {
            const int64_t gs = one_group ? (j_hi - j_lo + p->G)
                                         : std::min<int64_t>(p->group_spectra, j_hi - j_lo + p->G);
            zneed = (size_t)(gs + p->G) * p->npol * p->N;
        }
        st = ensure_scratch(p, zneed, part_floats);
        if (st != PFBS_OK) return st;
        sc = {p->Z, p->Zcap, p->part, p->partcap};
    }

    FrontArgs fa;
    memset(&fa, 0, sizeof fa);
    fa.fr = w.fr;
    fa.taps = p->taps;
    fa.g = p->gA;
    fa.N = p->N;
    fa.N1 = p->N1;
    fa.N2 = p->N2;
    fa.P = p->P;
    fa.ntiles = p->ntilesA;
    fa.ch = ch;
    fa.Z = sc.Z;
    fa.tw4 = p->tw4;
    fa.part = sc.part;
    fa.pt = tap_variant(p->pfb, p->P, p->tap_unroll == 1);
    if (!p->fourstep) {
        w.single = fa;
        w.single_chunks = (int)n_chunks;
    } else {
        BackArgs ba;
        memset(&ba, 0, sizeof ba);
        ba.Z = sc.Z;
        ba.g = p->gB;
        ba.N = p->N;
        ba.N1 = p->N1;
        ba.N2 = p->N2;
        ba.ntiles = p->ntilesB;
        ba.ch = ch;
        ba.part = sc.part;
        // groups of whole chunks whose intermediate fits the Z buffer
        const int64_t zlimit =
            one_group ? (j_hi - j_lo + p->G)
                      : std::min<int64_t>((int64_t)(sc.Zcap / ((size_t)p->npol * p->N)),
                                          std::max<int64_t>(p->group_spectra, p->G));
        int64_t g0 = gid_lo;
        while (g0 <= gid_hi) {
            int64_t gjs, gje, tjs, tje;
            chunk_span(p, g0, j_lo, j_hi, gjs, gje);
            int64_t g1 = g0;
            while (g1 + 1 <= gid_hi) {
                chunk_span(p, g1 + 1, j_lo, j_hi, tjs, tje);
                if (tje - gjs > zlimit) break;
                ++g1;
                gje = tje;
            }
            Group g;
            g.fa = fa;
            g.ba = ba;
            g.fa.ch.gid0 = g0;
            g.fa.jz0 = gjs;
            g.fa.sa0 = gjs;
            g.fa.sa1 = gje;
            // column pass: runs of ga spectra per workgroup.  One spectrum
            // per workgroup measured fastest (N = 2^15 and 2^19): the many
            // workgroups of one column tile then run side by side on one
            // XCD and share its taps and frames in L2.
            const int64_t ns = gje - gjs;
            g.fa.ga = p->ga_force > 0 ? p->ga_force : 1;
            g.fa.znt = p->znt;
            g.ba.znt = p->znt;
            g.fa.pair = p->pair;
            const int64_t run = (int64_t)g.fa.ga * (g.fa.pair ? 2 : 1);
            // items padded to a multiple of 8 for the XCD mapping (the
            // padding items find their spectra past the range and do nothing)
            g.na = (int)(((ns + run - 1) / run + 7) / 8 * 8);
            g.ba.ch.gid0 = g0;
            g.ba.jz0 = gjs;
            g.nc = (int)(g1 - g0 + 1);
            w.groups.push_back(g);
            g0 = g1 + 1;
        }
    }
    ReduceArgs &ra = w.ra;
    memset(&ra, 0, sizeof ra);
    ra.part = sc.part;
    ra.carried_in = p->carried[p->ccur];
    ra.carried_out = p->carried[p->ccur ^ 1];
    ra.out = d_dumps;
    ra.N = p->N;
    ra.N1 = p->N1;
    ra.N2 = p->fourstep ? p->N2 : 1;
    ra.n_prod = p->nprod;
    ra.n_int = p->n_int;
    ra.C = p->C;
    ra.G = p->G;
    ra.j_lo = j_lo;
    ra.j_hi = j_hi;
    ra.gid_lo = gid_lo;
    ra.gid_hi = gid_hi;
    ra.d_lo = j_lo / p->n_int;
    const int64_t d_hi = (j_hi - 1) / p->n_int;
    w.n_dumps = (int)(d_hi - ra.d_lo + 1);
    w.flip_carried = (d_hi + 1) * p->n_int > j_hi;  // an incomplete dump goes to carried_out
    return PFBS_OK;
}

pfbs_status launch_prepared(pfbs_plan *p, const Prepared &w, hipStream_t s, bool may_time = true) {
    // kernel timing creates events on demand; the allocation-free path never times
    const uint32_t timing = p->timing;
    if (!may_time) p->timing = 0;
    struct Restore {
        pfbs_plan *p;
        uint32_t t;
        ~Restore() { p->timing = t; }
    } restore{p, timing};
    if (w.any) {
        if (!p->fourstep) {
            PFBS_HIP(p, timed(p, 0, s, [&] { return launch_front(w.single, p->npol, p->pfb, true, p->prec_front, w.single_chunks, s); }));
        } else {
            for (const Group &g : w.groups) {
                PFBS_HIP(p, timed(p, 1, s, [&] { return launch_front(g.fa, p->npol, p->pfb, false, p->prec_front, g.na, s); }));
                PFBS_HIP(p, timed(p, 2, s, [&] { return launch_back(g.ba, p->npol, p->prec_back, g.nc, s); }));
            }
        }
        // the dump reduction and the tap-history copy share one launch
        if (w.hist)
            PFBS_HIP(p, timed(p, 3, s, [&] {
                return launch_reduce_history(w.ra, w.n_dumps, p->hist[p->hcur ^ 1], w.fr, w.F, p->P - 1,
                                             p->frame_bytes, s);
            }));
        else
            PFBS_HIP(p, timed(p, 3, s, [&] { return launch_reduce(w.ra, w.n_dumps, s); }));
        if ((p->out_stokes || p->out_shift) && w.nd_out > 0)
            PFBS_HIP(p, timed(p, 3, s, [&] {
                return launch_dump_format(w.ra.out, w.nd_out, p->N, p->nprod, p->out_stokes, p->out_shift, s);
            }));
    }
    if (w.hist && !w.any) {
        PFBS_HIP(p, timed(p, 4, s, [&] { return launch_history(p->hist[p->hcur ^ 1], w.fr, w.F, p->P - 1, p->frame_bytes, s); }));
    }
    return PFBS_OK;
}

void commit(pfbs_plan *p, const Prepared &w) {
    if (w.any && w.flip_carried) p->ccur ^= 1;
    if (w.hist) p->hcur ^= 1;
    p->frames_seen += w.F;
    p->spectra_done = w.j_hi;
    p->dumps_done += w.nd_out;
}

}  // namespace

extern "C" {

pfbs_status pfbs_execute(pfbs_plan *p, const void *d_block, int64_t n, float *d_dumps, int64_t cap,
                         int64_t *n_written, void *stream) {
    if (!n_written) return fail(PFBS_ERR_INVALID, "n_dumps_written is NULL");
    Prepared w;
    pfbs_status st = prepare(p, d_block, n, d_dumps, cap, false, w);
    if (st != PFBS_OK) return st;
    *n_written = 0;
    st = launch_prepared(p, w, (hipStream_t)stream);
    if (st != PFBS_OK) return st;
    commit(p, w);
    *n_written = w.nd_out;
    return PFBS_OK;
}

pfbs_status pfbs_execute_noalloc(pfbs_plan *p, const void *d_block, int64_t n, float *d_dumps, int64_t cap,
                                 int64_t *n_written, void *stream) {
    if (!n_written) return fail(PFBS_ERR_INVALID, "n_dumps_written is NULL");
    if (!plan_ok(p)) return fail(PFBS_ERR_STATE, "not a live plan");
    void *fixed = g_scratch_ptr[p->device];
    if (!fixed) return fail(PFBS_ERR_STATE, "no scratch address for device %d", p->device);
    Prepared w;
    pfbs_status st = prepare(p, d_block, n, d_dumps, cap, false, w, fixed, kNoAllocScratch);
    if (st != PFBS_OK) return st;
    *n_written = 0;
    st = launch_prepared(p, w, (hipStream_t)stream, false);
    if (st != PFBS_OK) return st;
    commit(p, w);
    *n_written = w.nd_out;
    return PFBS_OK;
}

pfbs_status pfbs_flush(pfbs_plan *p, float *d_partial, int64_t *n_spectra, void *stream) {
    if (!plan_ok(p)) return fail(PFBS_ERR_STATE, "not a live plan");
    if (p->poisoned) return fail(PFBS_ERR_STATE, "plan is poisoned");
    if (!d_partial || !n_spectra) return fail(PFBS_ERR_INVALID, "NULL argument");
    PFBS_HIP(p, hipSetDevice(p->device));
    const int64_t cnt = p->spectra_done - p->dumps_done * p->n_int;
    ReduceArgs ra;
    memset(&ra, 0, sizeof ra);
    ra.carried_in = p->carried[p->ccur];
    ra.out = d_partial;
    ra.N = p->N;
    ra.N1 = p->N1;
    ra.N2 = p->fourstep ? p->N2 : 1;
    ra.n_prod = p->nprod;
    ra.n_int = p->n_int;
    ra.C = p->C;
    ra.flush = 1;
    ra.have_carried = cnt > 0;
    PFBS_HIP(p, launch_reduce(ra, 1, (hipStream_t)stream));
    if (p->out_stokes || p->out_shift)
        PFBS_HIP(p, launch_dump_format(d_partial, 1, p->N, p->nprod, p->out_stokes, p->out_shift,
                                       (hipStream_t)stream));
    *n_spectra = cnt;
    return PFBS_OK;
}

pfbs_status pfbs_plan_reset(pfbs_plan *p) {
    if (!plan_ok(p)) return fail(PFBS_ERR_STATE, "not a live plan");
    hipError_t e = hipSetDevice(p->device);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(p, e, "reset");
    p->frames_seen = 0;
    p->spectra_done = 0;
    p->dumps_done = 0;
    p->hcur = 0;
    p->ccur = 0;
    p->poisoned = false;
    return PFBS_OK;
}

pfbs_status pfbs_debug_pfb(pfbs_plan *p, const void *d_block, int64_t n, float *d_y, int64_t ycap,
                           int64_t *n_spectra, void *stream) {
    pfbs_status st = check_block(p, d_block, n);
    if (st != PFBS_OK) return st;
    if (!n_spectra || !d_y) return fail(PFBS_ERR_INVALID, "NULL argument");
    int64_t j_lo, j_hi;
    block_spectra(p, n / p->N, j_lo, j_hi);
    if (ycap < j_hi - j_lo)
        return fail(PFBS_ERR_INVALID, "y capacity %lld < %lld spectra", (long long)ycap, (long long)(j_hi - j_lo));
    *n_spectra = j_hi - j_lo;
    if (j_hi == j_lo) return PFBS_OK;
    PFBS_HIP(p, hipSetDevice(p->device));
    Frames fr;
    fr.blk = (const uint8_t *)d_block;
    fr.hist = p->hist[p->hcur];
    fr.fs = p->frames_seen;
    fr.hf0 = p->frames_seen - (p->P - 1);
    PFBS_HIP(p, launch_debug_pfb(d_y, fr, p->taps, p->N, p->P, p->npol, p->pfb, j_lo, j_hi,
                                 (hipStream_t)stream));
    return PFBS_OK;
}

pfbs_status pfbs_plan_timing(pfbs_plan *p, int32_t enable) {
    return pfbs_plan_timing_kinds(p, enable ? (1u << PFBS_KERNEL_KINDS) - 1u : 0u);
}

pfbs_status pfbs_plan_timing_kinds(pfbs_plan *p, uint32_t kinds) {
    if (!plan_ok(p)) return fail(PFBS_ERR_STATE, "not a live plan");
    if (kinds >> PFBS_KERNEL_KINDS) return fail(PFBS_ERR_INVALID, "unknown kernel kind in mask 0x%x", kinds);
    p->timing = kinds;
    return PFBS_OK;
}

pfbs_status pfbs_plan_timing_read(pfbs_plan *p, double *ms, int64_t *launches, int32_t n) {
    if (!plan_ok(p)) return fail(PFBS_ERR_STATE, "not a live plan");
    if ((!ms || !launches) && n > 0) return fail(PFBS_ERR_INVALID, "NULL output arrays");
    PFBS_HIP(p, hipSetDevice(p->device));
    for (const auto &r : p->recs) {
        PFBS_HIP(p, hipEventSynchronize(p->ev_pool[r.i0 + 1]));
        float t = 0.f;
        PFBS_HIP(p, hipEventElapsedTime(&t, p->ev_pool[r.i0], p->ev_pool[r.i0 + 1]));
        if (r.kind < n) {
            ms[r.kind] += t;
            launches[r.kind] += 1;
        }
    }
    p->recs.clear();
    p->ev_used = 0;
    return PFBS_OK;
}

pfbs_status pfbs_debug_taps(pfbs_plan *p, float *d_out, void *stream) {
    if (!plan_ok(p)) return fail(PFBS_ERR_STATE, "not a live plan");
    if (!d_out) return fail(PFBS_ERR_INVALID, "d_out is NULL");
    PFBS_HIP(p, hipSetDevice(p->device));
    PFBS_HIP(p, hipMemcpyAsync(d_out, p->taps, (size_t)p->P * p->N * sizeof(float),
                               hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return PFBS_OK;
}

pfbs_status pfbs_debug_table(pfbs_plan *p, int32_t which, void *d_out, int64_t capacity_bytes, int64_t *bytes,
                             void *stream) {
    if (!plan_ok(p)) return fail(PFBS_ERR_STATE, "not a live plan");
    if (!bytes) return fail(PFBS_ERR_INVALID, "bytes is NULL");
    const void *src = nullptr;
    size_t n = 0;
    switch (which) {
    case PFBS_TABLE_TAPS: src = p->taps; n = (size_t)p->P * p->N * sizeof(float); break;
    case PFBS_TABLE_TW_FIRST: src = p->twA; n = (size_t)tw16_count(p->gA) * sizeof(float2); break;
    case PFBS_TABLE_TW_ROWS: src = p->twB; n = p->twB ? (size_t)tw16_count(p->gB) * sizeof(float2) : 0; break;
    case PFBS_TABLE_TW_ROWS_F64: src = p->twB64; n = p->twB64 ? (size_t)tw16_count(p->gB) * sizeof(double2) : 0; break;
    case PFBS_TABLE_TW_STEP: src = p->tw4; n = p->tw4 ? (size_t)p->N * sizeof(float2) : 0; break;
    case PFBS_TABLE_MFMA: src = p->mw; n = p->mw ? (size_t)64 * 4 * sizeof(uint4) : 0; break;
    default: return fail(PFBS_ERR_INVALID, "unknown table %d", which);
    }
    *bytes = (int64_t)n;
    if (n == 0 || !d_out) return PFBS_OK;
    if ((int64_t)n > capacity_bytes)
        return fail(PFBS_ERR_INVALID, "table needs %zu bytes, capacity %lld", n, (long long)capacity_bytes);
    PFBS_HIP(p, hipSetDevice(p->device));
    PFBS_HIP(p, hipMemcpyAsync(d_out, src, n, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return PFBS_OK;
}

// ---------------------------------------------------------------- batch ----

}  // extern "C"

namespace {

void batch_free(pfbs_batch *b) {
    for (pfbs_plan *p : b->plans) pfbs_plan_destroy(p);
    b->plans.clear();
    for (int k = 0; k < pfbs_batch::kTabRing; ++k) {
        if (b->gexec[k]) (void)hipGraphExecDestroy(b->gexec[k]);
        if (b->graph[k]) (void)hipGraphDestroy(b->graph[k]);
        if (b->copied[k]) (void)hipEventDestroy(b->copied[k]);
        if (b->done[k]) (void)hipEventDestroy(b->done[k]);
        if (b->h_tab[k]) (void)hipHostFree(b->h_tab[k]);
        if (b->d_tab[k]) (void)hipFree(b->d_tab[k]);
    }
    if (b->gstream) (void)hipStreamDestroy(b->gstream);
    if (b->cstream) (void)hipStreamDestroy(b->cstream);
}

// One kernel launch of a batched block.
struct BLaunch {
    const void *fn;
    int grid, threads;
    size_t lds;
    const void *table;
    int n;
    const void *table2;   // rows-and-single-passes kernel: the single-pass entries
    int n2;
    void *args[4];
    void **set_args() {
        args[0] = (void *)&table;
        args[1] = (void *)&n;
        args[2] = (void *)&table2;
        args[3] = (void *)&n2;
        return args;
    }
};

// Upper bounds on the workgroups of one sub-band's launches for a block of F
// frames (graph replays keep these grids; surplus workgroups exit at once).
int64_t max_chunks(const pfbs_plan *p, int64_t F) { return F / p->G + F / p->n_int + 3; }
int64_t max_dumps(const pfbs_plan *p, int64_t F) { return F / p->n_int + 2; }
int reduce_gx(const pfbs_plan *p) {
    return p->fourstep ? (int)((p->N2 / 32) * (p->N1 / 32)) : (int)((p->N + 255) / 256);  // k_reduce tiles
}
int hist_wg(const pfbs_plan *p) {
    return (int)std::min<int64_t>(1024, ((int64_t)(p->P - 1) * (p->frame_bytes / 16) + 255) / 256);
}
// Front-phase workgroups for `items` body blocks: two per workgroup (one per
// half) in groups of 8 workgroups, or one each for the two-spectra kernel.
int front_wg(int kind, int64_t items) {
    return kind == 2 ? (int)((items + 7) / 8 * 8) : (int)((items + 15) / 16 * 8);
}
// Row-phase tiles of a plan at the batch's tile size.
int batch_ntiles_b(const pfbs_plan *p, int tpb) { return (int)(p->N2 / (tpb / p->N1)); }
size_t batch_back_lds(const pfbs_plan *p, int tpb) {
    return back_lds_bytes(make_geo((int)p->N1, tpb), p->npol, p->prec_back);
}

}  // namespace

extern "C" {

pfbs_status pfbs_batch_create(pfbs_batch **out, const pfbs_plan_desc *descs, int32_t n) {
    if (!out) return fail(PFBS_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (!descs || n < 1 || n > kMaxBatch) return fail(PFBS_ERR_INVALID, "need 1..%d descriptions", kMaxBatch);
    for (int i = 0; i < n; ++i) {
        pfbs_status st = validate_desc(&descs[i]);
        if (st != PFBS_OK) return fail(st, "sub-band %d: %s", i, g_err.c_str());
        if (descs[i].n_pol != descs[0].n_pol) return fail(PFBS_ERR_INVALID, "all sub-bands need the same n_pol");
        if (descs[i].precision != PFBS_PREC_FP32 && descs[i].precision != PFBS_PREC_MIXED)
            return fail(PFBS_ERR_UNSUPPORTED, "sub-band %d: batched launches run the FP32 and MIXED paths", i);
        if (descs[i].output != PFBS_OUT_PRODUCTS || descs[i].fftshift != 0)
            return fail(PFBS_ERR_UNSUPPORTED, "sub-band %d: batched launches write the products in natural order", i);
    }
    pfbs_batch *b = new (std::nothrow) pfbs_batch();
    if (!b) return fail(PFBS_ERR_NOMEM, "host allocation");
    b->magic = kMagic;
    b->npol = descs[0].n_pol;
    b->tpb = 1024;
    pfbs_status st = PFBS_OK;
    for (int i = 0; i < n && st == PFBS_OK; ++i) {
        pfbs_plan *p = nullptr;
        st = pfbs_plan_create_ex(&p, &descs[i]);
        if (st != PFBS_OK) {
            std::string why = g_err;
            st = fail(st, "sub-band %d: %s", i, why.c_str());
            break;
        }
        b->plans.push_back(p);
        if (p->fourstep) b->tpb = std::max(b->tpb, back_tile((int)p->N1));
    }
    bool has_single = false;
    for (pfbs_plan *p : b->plans) has_single = has_single || !p->fourstep;
    // single passes go to the row phase (2048-point row tiles, whose
    // workgroup pair is one single-pass workgroup) unless a row is longer
    b->rows_single = st == PFBS_OK && has_single && b->tpb <= 2048;
    if (b->rows_single) b->tpb = 2048;
    if (st == PFBS_OK && !g_batch_ok[b->plans[0]->device])
        st = fail(PFBS_ERR_UNSUPPORTED, "the device refused the LDS size of the batched kernels");
    if (st == PFBS_OK) {
        // LDS of the two phase workgroups
        size_t lf = 0, lb = 0;
        const size_t rows_mul = b->rows_single ? 2 : 1;   // two row workgroups per workgroup
        for (pfbs_plan *p : b->plans) {
            if (!p->fourstep && b->rows_single) lb = std::max(lb, front_lds_bytes(p->gA, p->npol));
            else lf = std::max(lf, 2 * front_lds_bytes(p->gA, p->npol));
            if (p->fourstep) lb = std::max(lb, rows_mul * batch_back_lds(p, b->tpb));
        }
        if (lf > (size_t)kPairLds || lb > (size_t)kPairLds)
            st = fail(PFBS_ERR_UNSUPPORTED, "batched launches need %zu / %zu bytes of LDS (limit %d)", lf, lb,
                      kPairLds);
    }
    hipError_t e = hipSuccess;
    for (int k = 0; k < pfbs_batch::kTabRing && st == PFBS_OK && e == hipSuccess; ++k) {
        if ((e = hipMalloc((void **)&b->d_tab[k], sizeof(pfbs_batch::Tables))) == hipSuccess &&
            (e = hipHostMalloc((void **)&b->h_tab[k], sizeof(pfbs_batch::Tables), hipHostMallocDefault)) == hipSuccess &&
            (e = hipEventCreateWithFlags(&b->copied[k], hipEventDisableTiming)) == hipSuccess)
            e = hipEventCreateWithFlags(&b->done[k], hipEventDisableTiming);
    }
    // default-priority streams: table copies, and the one graphs are captured on
    if (st == PFBS_OK && e == hipSuccess && (e = hipStreamCreateWithFlags(&b->cstream, hipStreamNonBlocking)) == hipSuccess)
        e = hipStreamCreateWithFlags(&b->gstream, hipStreamNonBlocking);
    if (st == PFBS_OK && e != hipSuccess) st = hip_fail(nullptr, e, "batch resources");
    if (st != PFBS_OK) {
        batch_free(b);
        delete b;
        return st;
    }
    *out = b;
    return PFBS_OK;
}

pfbs_status pfbs_batch_execute(pfbs_batch *b, const void *const *d_blocks, const int64_t *n_samples,
                               float *const *d_dumps, const int64_t *caps, int64_t *n_dumps,
                               int32_t use_graph, void *stream) {
    if (!b || b->magic != kMagic) return fail(PFBS_ERR_STATE, "not a live batch");
    if (!d_blocks || !n_samples || !d_dumps || !caps || !n_dumps) return fail(PFBS_ERR_INVALID, "NULL argument");
    const int n = (int)b->plans.size();
    std::vector<Prepared> w(n);
    for (int i = 0; i < n; ++i) {
        pfbs_status st = prepare(b->plans[i], d_blocks[i], n_samples[i], d_dumps[i], caps[i], true, w[i]);
        if (st != PFBS_OK) return fail(st, "sub-band %d: %s", i, g_err.c_str());
    }
    pfbs_plan *p0 = b->plans[0];
    // ---- entry tables (buffer k; the host copy is free once its last upload is done)
    const int k = b->stage;
    hipError_t e = hipEventSynchronize(b->copied[k]);
    if (e != hipSuccess) return hip_fail(nullptr, e, "batch staging");
    // a graph replays fixed grids: recapture when the block sizes change
    const std::vector<int64_t> sizes(n_samples, n_samples + n);
    if (use_graph && b->gexec[k] && sizes != b->gsizes[k]) {
        (void)hipGraphExecDestroy(b->gexec[k]);
        (void)hipGraphDestroy(b->graph[k]);
        b->gexec[k] = nullptr;
        b->graph[k] = nullptr;
    }
    pfbs_batch::Tables &T = *b->h_tab[k];
    char *dbase = reinterpret_cast<char *>(b->d_tab[k]);
    const BatchFrontEntry *d_front =
        reinterpret_cast<const BatchFrontEntry *>(dbase + offsetof(pfbs_batch::Tables, front));
    const BatchBackEntry *d_back =
        reinterpret_cast<const BatchBackEntry *>(dbase + offsetof(pfbs_batch::Tables, back));
    const BatchTailEntry *d_tail =
        reinterpret_cast<const BatchTailEntry *>(dbase + offsetof(pfbs_batch::Tables, tail));
    std::vector<BLaunch> L;

    // ---- front phase: every sub-band's column pass, and its single pass
    // unless those run in the row phase.  Entries with the longest work per
    // workgroup first (single passes walk a whole chunk of spectra), so that
    // they start while the rest fill the machine.  Single passes that run in
    // the row phase sit at the end of the front table.
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    auto kind_of = [&](int i) { return !b->plans[i]->fourstep ? 0 : (w[i].any && w[i].groups[0].fa.pair ? 2 : 1); };
    auto rank = [&](int i) {
        const int k = kind_of(i);
        return k == 0 ? (b->rows_single ? 3 : 0) : (k == 2 ? 1 : 2);
    };
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        const int rx = rank(x), ry = rank(y);
        if (rx != ry) return rx < ry;
        return b->plans[x]->N > b->plans[y]->N;
    });
    int nf = 0, wf = 0, wf_max = 0;   // front-phase entries
    int ns = 0, ws = 0, ws_max = 0;   // single passes of the row phase
    size_t lds_f = 0, lds_s = 0;
    for (int i : order) {
        pfbs_plan *p = b->plans[i];
        const int64_t F = n_samples[i] / p->N;
        const int kind = kind_of(i);
        const bool in_rows = kind == 0 && b->rows_single;
        BatchFrontEntry &E = T.front[nf + ns];
        memset(&E, 0, sizeof E);
        E.kind = kind;
        E.pfb = p->pfb ? 1 : 0;
        E.L = (int)p->gA.L;
        int64_t items_max;
        const int64_t ga = std::max(1, p->ga_force);
        if (kind == 0) {
            if (w[i].any) {
                E.a = w[i].single;
                E.items = w[i].single_chunks;
            }
            items_max = max_chunks(p, F);
        } else {
            if (w[i].any) {
                E.a = w[i].groups[0].fa;
                E.items = w[i].groups[0].na * p->ntilesA;
            }
            const int64_t run = ga * (kind == 2 ? 2 : 1);
            items_max = p->ntilesA * (((F + run - 1) / run + 7) / 8 * 8);
        }
        E.pt = w[i].any ? E.a.pt : 0;
        if (in_rows) {
            // one single-pass workgroup per chunk, a whole row-phase workgroup
            E.wg0 = ws;
            E.wgn = w[i].any ? E.items : 0;
            ws += E.wgn;
            ws_max += (int)items_max;
            lds_s = std::max(lds_s, front_lds_bytes(p->gA, p->npol));
            ++ns;
        } else {
            E.wg0 = wf;
            E.wgn = w[i].any ? front_wg(kind, E.items) : 0;
            wf += E.wgn;
            wf_max += front_wg(kind, items_max);
            lds_f = std::max(lds_f, 2 * front_lds_bytes(p->gA, p->npol));
            ++nf;
        }
    }
    const bool front_single = !b->rows_single && std::any_of(b->plans.begin(), b->plans.end(),
                                                             [](const pfbs_plan *p) { return !p->fourstep; });
    if (nf > 0 && (wf > 0 || use_graph))
        L.push_back({batch_front_fn(b->npol, front_single), use_graph ? wf_max : wf, 2 * kTilePoints / 16 * b->npol,
                     lds_f, d_front, nf, nullptr, 0});

    // ---- row phase: every four-step sub-band's row pass at one tile size
    // (with the single passes: two row workgroups per workgroup)
    int nbk = 0, wb = 0, wb_max = 0;
    size_t lds_b = 0;
    for (int i : order) {
        pfbs_plan *p = b->plans[i];
        if (!p->fourstep) continue;
        const int64_t F = n_samples[i] / p->N;
        const int ntb = batch_ntiles_b(p, b->tpb);
        BatchBackEntry &E = T.back[nbk++];
        memset(&E, 0, sizeof E);
        E.L = (int)p->N1;
        E.prec = p->prec_back;
        E.wg0 = wb;
        int64_t items = 0;
        if (w[i].any) {
            E.a = w[i].groups[0].ba;
            E.a.ntiles = ntb;
            E.a.g.T = b->tpb / (int)p->N1;
            items = (int64_t)w[i].groups[0].nc * ntb;
        }
        E.items = (int)items;
        const int64_t items_max = ntb * max_chunks(p, F);
        if (b->rows_single) {
            E.wgn = (int)((items + 15) / 16 * 8);
            wb_max += (int)((items_max + 15) / 16 * 8);
            lds_b = std::max(lds_b, 2 * batch_back_lds(p, b->tpb));
        } else {
            E.wgn = (int)items;
            wb_max += (int)items_max;
            lds_b = std::max(lds_b, batch_back_lds(p, b->tpb));
        }
        wb += E.wgn;
    }
    if (b->rows_single) {
        if (wb + ws > 0 || use_graph)
            L.push_back({batch_rows_single_fn(b->npol), use_graph ? wb_max + ws_max : wb + ws,
                         2 * b->tpb / 16 * b->npol, std::max(lds_b, lds_s), d_back, nbk, d_front + nf, ns});
    } else if (nbk > 0 && (wb > 0 || use_graph)) {
        L.push_back({batch_back_fn(b->npol, b->tpb), use_graph ? wb_max : wb, b->tpb / 16 * b->npol, lds_b, d_back,
                     nbk, nullptr, 0});
    }

    // ---- tail: dump reductions and history copies
    int ntl = 0, wt = 0, wt_max = 0;
    for (int i = 0; i < n; ++i) {
        pfbs_plan *p = b->plans[i];
        const int64_t F = n_samples[i] / p->N;
        BatchTailEntry &R = T.tail[ntl++];
        memset(&R, 0, sizeof R);
        R.kind = 0;
        R.gx = reduce_gx(p);
        R.wg0 = wt;
        if (w[i].any) {
            R.r = w[i].ra;
            R.gy = w[i].n_dumps;
            R.wgn = R.gx * R.gy * p->nprod;
        }
        wt += R.wgn;
        wt_max += (int)(R.gx * max_dumps(p, F) * p->nprod);
        if (w[i].hist) {
            BatchTailEntry &H = T.tail[ntl++];
            memset(&H, 0, sizeof H);
            H.kind = 1;
            H.hdst = p->hist[p->hcur ^ 1];
            H.fr = w[i].fr;
            H.F = w[i].F;
            H.H = p->P - 1;
            H.frame_vec = p->frame_bytes / 16;
            H.wg0 = wt;
            H.wgn = hist_wg(p);
            wt += H.wgn;
            wt_max += H.wgn;
        }
    }
    if (wt > 0 || use_graph) L.push_back({batch_tail_fn(), use_graph ? wt_max : wt, 256, 0, d_tail, ntl, nullptr, 0});

    hipStream_t cs = (hipStream_t)stream;
    PFBS_HIP(p0, hipSetDevice(p0->device));
    // upload on the copy stream once the kernels that last read this device
    // buffer are done; the caller's stream waits only for the upload (done
    // long before, while it ran the blocks in between)
    PFBS_HIP(p0, hipStreamWaitEvent(b->cstream, b->done[k], 0));
    PFBS_HIP(p0, hipMemcpyAsync(b->d_tab[k], &T, sizeof T, hipMemcpyHostToDevice, b->cstream));
    PFBS_HIP(p0, hipEventRecord(b->copied[k], b->cstream));
    PFBS_HIP(p0, hipStreamWaitEvent(cs, b->copied[k], 0));
    b->launches = 0;
    if (!use_graph) {
        for (BLaunch &x : L) {
            if (x.grid <= 0) continue;
            PFBS_HIP(p0, hipLaunchKernel(x.fn, dim3(x.grid), dim3(x.threads), x.set_args(), x.lds, cs));
            ++b->launches;
        }
    } else {
        if (!b->gexec[k]) {
            hipStream_t s = b->gstream;
            PFBS_HIP(p0, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            hipError_t le = hipSuccess;
            for (BLaunch &x : L) {
                if (le == hipSuccess)
                    le = hipLaunchKernel(x.fn, dim3(x.grid > 0 ? x.grid : 1), dim3(x.threads), x.set_args(), x.lds, s);
            }
            hipGraph_t g = nullptr;
            hipError_t ce = hipStreamEndCapture(s, &g);
            if (le != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return hip_fail(p0, le, "batch capture launch");
            }
            if (ce != hipSuccess) return hip_fail(p0, ce, "batch capture");
            b->graph[k] = g;
            PFBS_HIP(p0, hipGraphInstantiate(&b->gexec[k], b->graph[k], nullptr, nullptr, 0));
            b->gsizes[k] = sizes;
        }
        // captured on the batch's own stream, replayed on the caller's
        PFBS_HIP(p0, hipGraphLaunch(b->gexec[k], cs));
        b->launches = (int)L.size();
    }
    PFBS_HIP(p0, hipEventRecord(b->done[k], cs));
    b->stage = (b->stage + 1) % pfbs_batch::kTabRing;
    for (int i = 0; i < n; ++i) {
        commit(b->plans[i], w[i]);
        n_dumps[i] = w[i].nd_out;
    }
    return PFBS_OK;
}

int32_t pfbs_batch_launches(const pfbs_batch *b) {
    if (!b || b->magic != kMagic) return -1;
    return b->launches;
}

pfbs_status pfbs_batch_destroy(pfbs_batch *b) {
    if (!b) return PFBS_OK;
    if (b->magic != kMagic) return fail(PFBS_ERR_STATE, "not a live batch");
    if (!b->plans.empty()) {
        (void)hipSetDevice(b->plans[0]->device);
        (void)hipDeviceSynchronize();
    }
    batch_free(b);
    b->magic = kDead;
    delete b;
    return PFBS_OK;
}

pfbs_plan *pfbs_batch_plan(pfbs_batch *b, int32_t i) {
    if (!b || b->magic != kMagic || i < 0 || i >= (int32_t)b->plans.size()) return nullptr;
    return b->plans[i];
}

}  // extern "C"

namespace pfbs {

pfbs_status validate_desc_quiet(const pfbs_plan_desc *d) {
    const std::string keep = g_err;
    const pfbs_status st = validate_desc(d);
    g_err = keep;
    return st;
}

}  // namespace pfbs
