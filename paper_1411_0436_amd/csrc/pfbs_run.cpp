// pfbs_run: a plain C-ABI driver of the spectrometer, for profilers that must
// watch a program without an interpreter in between (hardware counters), and
// as an example of the boundary used from C/C++.
//
//   pfbs_run N P mode n_pol n_int block_samples blocks steps [precision [split_n2 [chunk [col_pair]]]]
//       mode 0 = PFB (Hann-windowed sinc), 1 = direct.  Allocates `blocks`
//       device blocks of block_samples time samples filled with seeded
//       pseudo-random int8 values, runs one untimed pass and then `steps`
//       passes over all blocks through pfbs_execute, and prints one line of
//       JSON: complex samples per second and the per-kernel times from the
//       plan's own HIP events.
//   pfbs_run --copy MiB
//       one device-to-device hipMemcpy of MiB mebibytes (repeated 5 times):
//       the reference transfer that scales the byte counters.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../../include/pfbspec.h"

#define CHECK_HIP(x)                                                                   \
    do {                                                                               \
        hipError_t e_ = (x);                                                           \
        if (e_ != hipSuccess) {                                                        \
            fprintf(stderr, "%s:%d %s: %s\n", __FILE__, __LINE__, #x, hipGetErrorString(e_)); \
            return 1;                                                                  \
        }                                                                              \
    } while (0)
#define CHECK_PFBS(x)                                                                  \
    do {                                                                               \
        pfbs_status s_ = (x);                                                          \
        if (s_ != PFBS_OK) {                                                           \
            fprintf(stderr, "%s:%d %s: status %d: %s\n", __FILE__, __LINE__, #x, (int)s_, \
                    pfbs_last_error());                                                \
            return 1;                                                                  \
        }                                                                              \
    } while (0)

static int run_copy(long long mib) {
    const size_t n = (size_t)mib << 20;
    void *a = nullptr, *b = nullptr;
    CHECK_HIP(hipMalloc(&a, n));
    CHECK_HIP(hipMalloc(&b, n));
    CHECK_HIP(hipMemset(a, 1, n));
    for (int i = 0; i < 5; ++i) CHECK_HIP(hipMemcpy(b, a, n, hipMemcpyDeviceToDevice));
    CHECK_HIP(hipDeviceSynchronize());
    printf("{\"copy_bytes_read\": %zu, \"copy_bytes_written\": %zu, \"launches\": 5}\n", n, n);
    CHECK_HIP(hipFree(a));
    CHECK_HIP(hipFree(b));
    return 0;
}

int main(int argc, char **argv) {
    if (argc == 3 && strcmp(argv[1], "--copy") == 0) return run_copy(atoll(argv[2]));
    if (argc < 9) {
        fprintf(stderr, "usage: %s N P mode n_pol n_int block_samples blocks steps "
                        "[precision [split_n2 [chunk [col_pair]]]]\n"
                        "       %s --copy MiB\n", argv[0], argv[0]);
        return 2;
    }
    pfbs_plan_desc d;
    memset(&d, 0, sizeof d);
    d.N = atoll(argv[1]);
    d.P = atoi(argv[2]);
    d.mode = atoi(argv[3]);
    d.n_pol = atoi(argv[4]);
    d.n_int = atoll(argv[5]);
    const long long B = atoll(argv[6]);
    const int nblk = atoi(argv[7]), steps = atoi(argv[8]);
    d.precision = argc > 9 ? atoi(argv[9]) : 0;
    d.split_n2 = argc > 10 ? atoll(argv[10]) : 0;
    d.chunk = argc > 11 ? atoi(argv[11]) : 0;
    d.col_pair = argc > 12 ? atoi(argv[12]) : 0;
    d.window = PFBS_WINDOW_HANN_SINC;
    d.device = -1;
    if (nblk < 1 || steps < 1 || B <= 0) {
        fprintf(stderr, "blocks, steps and block_samples must be positive\n");
        return 2;
    }
    pfbs_plan *plan = nullptr;
    CHECK_PFBS(pfbs_plan_create_ex(&plan, &d));

    // seeded pseudo-random int8 samples (xorshift64*), one host buffer per block
    const size_t bytes = (size_t)B * 2 * d.n_pol;
    std::vector<void *> blk(nblk, nullptr);
    std::vector<uint8_t> host(bytes);
    uint64_t st = 0x9E3779B97F4A7C15ull;
    for (int b = 0; b < nblk; ++b) {
        for (size_t i = 0; i < bytes; ++i) {
            st ^= st >> 12;
            st ^= st << 25;
            st ^= st >> 27;
            host[i] = (uint8_t)((st * 0x2545F4914F6CDD1Dull) >> 56);
        }
        CHECK_HIP(hipMalloc(&blk[b], bytes));
        CHECK_HIP(hipMemcpy(blk[b], host.data(), bytes, hipMemcpyHostToDevice));
    }
    const int n_prod = d.n_pol == 2 ? 4 : 1;
    const long long cap = B / d.N / d.n_int + 2;
    float *dumps = nullptr;
    CHECK_HIP(hipMalloc((void **)&dumps, (size_t)cap * n_prod * d.N * sizeof(float)));
    hipStream_t s;
    CHECK_HIP(hipStreamCreate(&s));
    int64_t nd = 0;
    for (int b = 0; b < nblk; ++b) CHECK_PFBS(pfbs_execute(plan, blk[b], B, dumps, cap, &nd, s));
    CHECK_HIP(hipStreamSynchronize(s));
    CHECK_PFBS(pfbs_plan_timing(plan, 1));
    hipEvent_t e0, e1;
    CHECK_HIP(hipEventCreate(&e0));
    CHECK_HIP(hipEventCreate(&e1));
    CHECK_HIP(hipEventRecord(e0, s));
    for (int i = 0; i < steps; ++i)
        for (int b = 0; b < nblk; ++b) CHECK_PFBS(pfbs_execute(plan, blk[b], B, dumps, cap, &nd, s));
    CHECK_HIP(hipEventRecord(e1, s));
    CHECK_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    CHECK_HIP(hipEventElapsedTime(&ms, e0, e1));
    double kms[PFBS_KERNEL_KINDS];
    int64_t kn[PFBS_KERNEL_KINDS];
    memset(kms, 0, sizeof kms);
    memset(kn, 0, sizeof kn);
    CHECK_PFBS(pfbs_plan_timing_read(plan, kms, kn, PFBS_KERNEL_KINDS));
    const char *names[PFBS_KERNEL_KINDS] = {"single_pass", "column_pass", "row_pass", "dump_reduce",
                                            "tap_history"};
    const double samples = (double)steps * nblk * B * d.n_pol;
    printf("{\"Gsamples_s\": %.3f, \"ms_per_step\": %.4f, \"kernel_ms\": {", samples / (ms * 1e-3) / 1e9,
           ms / steps);
    bool first = true;
    for (int k = 0; k < PFBS_KERNEL_KINDS; ++k) {
        if (!kn[k]) continue;
        printf("%s\"%s\": %.5f", first ? "" : ", ", names[k], kms[k] / kn[k]);
        first = false;
    }
    printf("}}\n");
    for (void *p : blk) CHECK_HIP(hipFree(p));
    CHECK_HIP(hipFree(dumps));
    CHECK_HIP(hipStreamDestroy(s));
    CHECK_PFBS(pfbs_plan_destroy(plan));
    return 0;
}
