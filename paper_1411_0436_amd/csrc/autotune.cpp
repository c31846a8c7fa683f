// Autotuner for the speed-only plan fields (split of the two-pass FFT, chunk
// length of the partial integrations, spectra per column-pass workgroup,
// streaming intermediate).  Every candidate computes the same spectra; they
// differ only in how the work is cut and scheduled on the device.  Candidates
// are timed with HIP events on one synthetic device block and the fastest is
// kept, optionally in a plain-text cache file (PFBS_TUNE_CACHE).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/pfbspec.h"
#include "pfbs_internal.h"

namespace {

std::mutex g_cache_mu;

bool pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

std::string device_arch() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return "unknown";
    hipDeviceProp_t pr;
    if (hipGetDeviceProperties(&pr, dev) != hipSuccess) return "unknown";
    std::string a = pr.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

#ifndef PFBS_SOURCE_DIGEST
#define PFBS_SOURCE_DIGEST "unknown"
#endif

struct Line {
    std::string arch, version;
    long long N, n_int, block, split;
    int P, mode, npol, prec, chunk, col_run, stream_z, tap_unroll, col_pair;
    double sps;
};

bool parse(const char *s, Line &l) {
    char tag[32], arch[64], ver[64];
    int n = sscanf(s, "%31s %63s %63s %lld %d %d %d %lld %d %lld %lld %d %d %d %d %d %lf", tag, arch, ver, &l.N,
                   &l.P, &l.mode, &l.npol, &l.n_int, &l.prec, &l.block, &l.split, &l.chunk, &l.col_run,
                   &l.stream_z, &l.tap_unroll, &l.col_pair, &l.sps);
    if (n != 17 || strcmp(tag, "pfbs-tune-v3") != 0) return false;
    l.arch = arch;
    l.version = ver;
    return true;
}

bool same_shape(const Line &l, const std::string &arch, const pfbs_plan_desc *d) {
    return l.arch == arch && l.version == PFBS_SOURCE_DIGEST && l.N == d->N && l.P == d->P && l.mode == d->mode &&
           l.npol == d->n_pol &&
           l.n_int == d->n_int && l.prec == d->precision;
}

bool cache_find(const pfbs_plan_desc *d, Line &best) {
    const char *path = getenv("PFBS_TUNE_CACHE");
    if (!path || !*path) return false;
    std::lock_guard<std::mutex> lk(g_cache_mu);
    FILE *f = fopen(path, "r");
    if (!f) return false;
    const std::string arch = device_arch();
    char buf[512];
    bool found = false;
    while (fgets(buf, sizeof buf, f)) {
        Line l;
        if (parse(buf, l) && same_shape(l, arch, d)) {  // newest matching line wins
            best = l;
            found = true;
        }
    }
    fclose(f);
    return found;
}

void cache_append(const pfbs_plan_desc *d, int64_t block, const pfbs_plan_desc *b, double sps) {
    const char *path = getenv("PFBS_TUNE_CACHE");
    if (!path || !*path) return;
    std::lock_guard<std::mutex> lk(g_cache_mu);
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "pfbs-tune-v3 %s %s %lld %d %d %d %lld %d %lld %lld %d %d %d %d %d %.6e\n", device_arch().c_str(),
            PFBS_SOURCE_DIGEST, (long long)d->N, d->P, d->mode, d->n_pol, (long long)d->n_int, d->precision,
            (long long)block, (long long)b->split_n2, b->chunk, b->col_run, b->stream_z, b->tap_unroll, b->col_pair, sps);
    fclose(f);
}

// Valid column lengths of the two-pass FFT for N (mirrors the plan's checks).
// Column lengths worth timing: every one the kernels support.
std::vector<int64_t> splits_for(int64_t N) {
    std::vector<int64_t> v;
    if (N <= pfbs::kMaxSinglePass) {
        v.push_back(0);
        return v;
    }
    for (int64_t n2 = 64; n2 <= 512; n2 *= 2) {
        const int64_t n1 = N / n2;
        if (n1 < 32 || n1 > pfbs::kMaxSinglePass) continue;
        const int tb = pfbs::back_tile_points(n1);
        if (n1 % (pfbs::kTilePoints / n2) == 0 && n2 % (tb / n1) == 0) v.push_back(n2);
    }
    return v;
}

// Time one candidate: average seconds per block over `reps` passes over the
// nb blocks (consecutive blocks of one stream) after `warm` untimed passes.
// Returns < 0 when the candidate cannot be created.
double time_candidate(const pfbs_plan_desc *c, const uint8_t *d_blocks, int nb, int64_t n, float *d_dumps,
                      int64_t cap, hipStream_t s, int warm, int reps) {
    pfbs_plan *p = nullptr;
    if (pfbs_plan_create_ex(&p, c) != PFBS_OK) return -1.0;
    hipEvent_t e0, e1;
    double t = -1.0;
    if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
        int64_t nd = 0;
        bool ok = true;
        const size_t bytes = (size_t)n * 2 * c->n_pol;
        for (int i = 0; i < warm * nb && ok; ++i)
            ok = pfbs_execute(p, d_blocks + (size_t)(i % nb) * bytes, n, d_dumps, cap, &nd, s) == PFBS_OK;
        ok = ok && hipEventRecord(e0, s) == hipSuccess;
        for (int i = 0; i < reps * nb && ok; ++i)
            ok = pfbs_execute(p, d_blocks + (size_t)(i % nb) * bytes, n, d_dumps, cap, &nd, s) == PFBS_OK;
        ok = ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
        float ms = 0.f;
        if (ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess) t = ms * 1e-3 / (reps * nb);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    pfbs_plan_destroy(p);
    return t;
}

}  // namespace

namespace pfbs {

pfbs_status tune_lookup(const pfbs_plan_desc *desc, bool measure_if_missing, pfbs_plan_desc *out) {
    *out = *desc;
    out->tune = 0;
    Line l;
    if (cache_find(desc, l)) {
        out->split_n2 = l.split;
        out->chunk = l.chunk;
        out->col_run = l.col_run;
        out->stream_z = l.stream_z;
        out->tap_unroll = l.tap_unroll;
        out->col_pair = l.col_pair;
        return PFBS_OK;
    }
    if (!measure_if_missing) return PFBS_OK;
    pfbs_plan_desc shape = *out;
    return pfbs_autotune(&shape, 0, 0, out, nullptr);
}

}  // namespace pfbs

extern "C" pfbs_status pfbs_autotune(const pfbs_plan_desc *desc, int64_t block_samples,
                                     int32_t max_candidates, pfbs_plan_desc *best,
                                     double *best_samples_per_s) {
    if (!desc || !best) return PFBS_ERR_INVALID;
    pfbs_plan_desc base = *desc;
    base.tune = 0;
    if (!pow2(base.N)) return PFBS_ERR_INVALID;
    int64_t n = block_samples > 0 ? block_samples : (int64_t(1) << 24);
    if (n % base.N != 0 || n < base.N) return PFBS_ERR_INVALID;
    // enough frames for a few spectra per block
    const int64_t need = (int64_t)(base.mode == PFBS_MODE_DIRECT ? 1 : base.P) + 3;
    if (n / base.N < need) n = need * base.N;
    if (base.device >= 0 && hipSetDevice(base.device) != hipSuccess) return PFBS_ERR_DEVICE;

    // candidate list: every valid split x chunk x run length; streaming off
    std::vector<pfbs_plan_desc> cands;
    const std::vector<int64_t> splits = splits_for(base.N);
    const bool four = base.N > pfbs::kMaxSinglePass;
    const int chunks[] = {8, 16, 32, 64};
    const int runs[] = {1, 2, 4};
    // the tap loop's form matters only with the filter at 4 or 8 taps
    const bool unrollable = base.mode == PFBS_MODE_PFB && (base.P == 4 || base.P == 8);
    for (int64_t sp : splits)
        for (int ch : chunks)
            for (int r = 0; r < (four ? 3 : 1); ++r)
                for (int u = unrollable ? 1 : 0; u <= (unrollable ? 2 : 0); ++u) {
                    pfbs_plan_desc c = base;
                    c.split_n2 = sp;
                    c.chunk = ch;
                    c.col_run = four ? runs[r] : 0;
                    c.stream_z = 0;
                    c.group_bytes = 0;
                    c.tap_unroll = u;
                    cands.push_back(c);
                }
    if (four) {  // streaming intermediate, at the default split
        pfbs_plan_desc c = base;
        c.stream_z = 1;
        c.col_run = 1;
        cands.push_back(c);
    }
    if (max_candidates > 0 && (int)cands.size() > max_candidates) cands.resize(max_candidates);

    const size_t bytes = (size_t)n * 2 * base.n_pol;
    // enough distinct blocks (at least 512 MB, at most 16) that the input
    // streams from HBM as in a real run instead of staying in the caches
    const int nb = (int)std::min<size_t>(16, std::max<size_t>(1, ((size_t)512 << 20) / bytes));
    void *d_block = nullptr;
    float *d_dumps = nullptr;
    const int64_t nprod = base.n_pol == 2 ? 4 : 1;
    const int64_t cap = n / base.N + 1;  // at most one dump per spectrum
    hipStream_t s = nullptr;
    pfbs_status rs = PFBS_OK;
    if (hipMalloc(&d_block, bytes * nb) != hipSuccess ||
        hipMalloc((void **)&d_dumps, (size_t)cap * nprod * base.N * sizeof(float)) != hipSuccess ||
        hipStreamCreate(&s) != hipSuccess) {
        rs = PFBS_ERR_NOMEM;
    }
    double best_t = -1.0;
    pfbs_plan_desc winner = base;
    if (rs == PFBS_OK && pfbs::launch_synth((uint32_t *)d_block, (long long)(bytes * nb / 4), 0x5eedu, s) != hipSuccess)
        rs = PFBS_ERR_DEVICE;
    if (rs == PFBS_OK) {
        for (const pfbs_plan_desc &c : cands) {
            const double t = time_candidate(&c, (const uint8_t *)d_block, nb, n, d_dumps, cap, s, 1, 2);
            if (t > 0 && (best_t < 0 || t < best_t)) {
                best_t = t;
                winner = c;
            }
        }
        if (best_t < 0) rs = PFBS_ERR_DEVICE;
    }
    if (s) (void)hipStreamDestroy(s);
    if (d_block) (void)hipFree(d_block);
    if (d_dumps) (void)hipFree(d_dumps);
    if (rs != PFBS_OK) return rs;
    const double sps = (double)n * base.n_pol / best_t;
    winner.tune = 0;
    *best = winner;
    if (best_samples_per_s) *best_samples_per_s = sps;
    cache_append(&base, n, &winner, sps);
    return PFBS_OK;
}
