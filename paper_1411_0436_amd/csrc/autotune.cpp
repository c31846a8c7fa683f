// Autotuner for the speed-only plan fields: the radix split of the two-pass
// FFT (column length), the column pass's workgroup form (one or two spectra
// per step: 8 or 16 waves), the pre-filter's tap loop, the row pass's tile
// width (rows per workgroup step, hence its waves per workgroup), the chunk
// length of the partial integrations, spectra per column-pass workgroup and
// the streaming intermediate.  Every candidate computes the same spectra to
// the precision's accuracy (splits are limited by split_keeps_accuracy); they
// differ in how the work is cut and scheduled on the device.  Candidates are
// timed with HIP events on synthetic device blocks in a coordinate search
// (each field in turn, the others at their best so far) and the fastest is
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
    int P, mode, npol, prec, chunk, col_run, stream_z, tap_unroll, col_pair, row_tile;
    double sps;
};

bool parse(const char *s, Line &l) {
    char tag[32], arch[64], ver[64];
    int n = sscanf(s, "%31s %63s %63s %lld %d %d %d %lld %d %lld %lld %d %d %d %d %d %d %lf", tag, arch, ver, &l.N,
                   &l.P, &l.mode, &l.npol, &l.n_int, &l.prec, &l.block, &l.split, &l.chunk, &l.col_run,
                   &l.stream_z, &l.tap_unroll, &l.col_pair, &l.row_tile, &l.sps);
    if (n != 18 || strcmp(tag, "pfbs-tune-v4") != 0) return false;
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
    fprintf(f, "pfbs-tune-v4 %s %s %lld %d %d %d %lld %d %lld %lld %d %d %d %d %d %d %.6e\n", device_arch().c_str(),
            PFBS_SOURCE_DIGEST, (long long)d->N, d->P, d->mode, d->n_pol, (long long)d->n_int, d->precision,
            (long long)block, (long long)b->split_n2, b->chunk, b->col_run, b->stream_z, b->tap_unroll, b->col_pair,
            b->row_tile, sps);
    fclose(f);
}

// Column lengths worth timing: every one the kernels support for N that
// keeps the precision's accuracy (0 = one pass).
std::vector<int64_t> splits_for(int64_t N, int precision) {
    std::vector<int64_t> v;
    if (N <= pfbs::kMaxSinglePass) {
        v.push_back(0);
        return v;
    }
    for (int64_t n2 = 64; n2 <= 512; n2 *= 2) {
        const int64_t n1 = N / n2;
        if (n1 < 32 || n1 > pfbs::kMaxSinglePass) continue;
        const int tb = pfbs::back_tile_points(n1);
        if (n1 % (pfbs::kTilePoints / n2) == 0 && n2 % (tb / n1) == 0 &&
            pfbs::split_keeps_accuracy(N, precision, n2))
            v.push_back(n2);
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
        out->row_tile = l.row_tile;
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

    // the fields searched, each with its values (0: the plan's automatic choice)
    const bool four = base.N > pfbs::kMaxSinglePass;
    const bool unrollable = base.mode == PFBS_MODE_PFB && (base.P == 4 || base.P == 8);
    struct Field {
        int64_t pfbs_plan_desc::*wide;
        int32_t pfbs_plan_desc::*narrow;
        std::vector<int64_t> values;
    };
    std::vector<Field> fields;
    if (four) {
        fields.push_back({&pfbs_plan_desc::split_n2, nullptr, splits_for(base.N, base.precision)});
        if (base.mode == PFBS_MODE_PFB) fields.push_back({nullptr, &pfbs_plan_desc::col_pair, {2, 1}});
    }
    if (unrollable) fields.push_back({nullptr, &pfbs_plan_desc::tap_unroll, {2, 1}});
    if (four) fields.push_back({nullptr, &pfbs_plan_desc::row_tile, {0, 2048, 4096}});
    fields.push_back({nullptr, &pfbs_plan_desc::chunk, {4, 8, 16, 32, 64}});
    if (four) {
        fields.push_back({nullptr, &pfbs_plan_desc::col_run, {1, 2, 4}});
        fields.push_back({nullptr, &pfbs_plan_desc::stream_z, {0, 1}});
    }
    auto get = [](const pfbs_plan_desc &d, const Field &f) -> int64_t { return f.wide ? d.*f.wide : d.*f.narrow; };
    auto set = [](pfbs_plan_desc &d, const Field &f, int64_t v) {
        if (f.wide) d.*f.wide = v;
        else d.*f.narrow = (int32_t)v;
    };
    base.group_bytes = 0;
    if (four && base.split_n2 == 0) base.split_n2 = pfbs::default_split(base.N);
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
    int timed_n = 0;
    if (rs == PFBS_OK && pfbs::launch_synth((uint32_t *)d_block, (long long)(bytes * nb / 4), 0x5eedu, s) != hipSuccess)
        rs = PFBS_ERR_DEVICE;
    auto try_cand = [&](const pfbs_plan_desc &c) {
        if (max_candidates > 0 && timed_n >= max_candidates) return;
        pfbs_plan_desc v = c;
        if (pfbs::validate_desc_quiet(&v) != PFBS_OK) return;  // e.g. a row tile shorter than the rows
        ++timed_n;
        const double t = time_candidate(&v, (const uint8_t *)d_block, nb, n, d_dumps, cap, s, 1, 3);
        if (t > 0 && (best_t < 0 || t < best_t)) {
            best_t = t;
            winner = v;
        }
    };
    if (rs == PFBS_OK) {
        // an untimed run of the starting point first: the device's clocks and
        // caches settle before any candidate is compared, so that the first
        // one timed is not the one that pays for it
        {
            pfbs_plan_desc v = base;
            if (pfbs::validate_desc_quiet(&v) == PFBS_OK)
                (void)time_candidate(&v, (const uint8_t *)d_block, nb, n, d_dumps, cap, s, 2, 1);
        }
        try_cand(base);
        for (const Field &f : fields) {
            const pfbs_plan_desc cur = winner;
            for (int64_t v : f.values) {
                if (v == get(cur, f)) continue;
                pfbs_plan_desc c = cur;
                set(c, f, v);
                try_cand(c);
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
