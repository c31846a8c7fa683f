// Host-fed streaming: a plan fed from host memory through a ring of device
// buffers.  The paper's loop copies each block host-to-device, computes, and
// copies the results back (Section 4, algorithm list), and names the copies
// as the cost that dominates small transforms (Section 5), with streams as
// the remedy.  Here three streams overlap them: block i+1 travels over PCIe
// while block i is computed and block i-1's dumps travel back.
//
//   copy-in stream : H2D of the block into slot k            -> ev_in[k]
//   compute stream : waits ev_in[k], pfbs_execute            -> ev_comp[k]
//   copy-out stream: waits ev_comp[k], D2H of the dumps      -> ev_out[k]
//
// A push that reuses slot k first waits (on the host) for ev_out[k] of the
// push `depth` places earlier, which also tells the caller that push's host
// buffers are free.  All streams have the default priority.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/pfbspec.h"
#include "pfbs_internal.h"

struct pfbs_hstream {
    uint32_t magic;
    pfbs_plan *plan;
    pfbs_plan_info info;
    int device;
    int64_t max_block;
    int depth;
    int64_t slot_cap;                // dumps a slot's device buffer holds
    std::vector<void *> d_blk;
    std::vector<float *> d_dumps;
    std::vector<hipEvent_t> ev_in, ev_comp, ev_out;
    std::vector<bool> used;
    hipStream_t s_in, s_comp, s_out;
    int64_t pushes;
};

namespace {

constexpr uint32_t kLive = 0x48535452u;  // "HSTR"

pfbs_status err(pfbs_status st, const char *what, hipError_t e = hipSuccess) {
    char buf[400];
    if (e != hipSuccess) snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    else snprintf(buf, sizeof buf, "%s", what);
    return pfbs::record_error(st, buf);
}

void release(pfbs_hstream *s) {
    if (s->device >= 0) (void)hipSetDevice(s->device);
    for (hipStream_t st : {s->s_in, s->s_comp, s->s_out})
        if (st) (void)hipStreamSynchronize(st);
    for (void *p : s->d_blk)
        if (p) (void)hipFree(p);
    for (float *p : s->d_dumps)
        if (p) (void)hipFree(p);
    for (auto *v : {&s->ev_in, &s->ev_comp, &s->ev_out})
        for (hipEvent_t e : *v)
            if (e) (void)hipEventDestroy(e);
    for (hipStream_t st : {s->s_in, s->s_comp, s->s_out})
        if (st) (void)hipStreamDestroy(st);
    if (s->plan) pfbs_plan_destroy(s->plan);
    s->plan = nullptr;
}

}  // namespace

extern "C" {

pfbs_status pfbs_host_alloc(void **out, int64_t bytes) {
    if (!out) return err(PFBS_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (bytes <= 0) return err(PFBS_ERR_INVALID, "bytes must be positive");
    hipError_t e = hipHostMalloc(out, (size_t)bytes, hipHostMallocDefault);
    if (e != hipSuccess) {
        *out = nullptr;
        return err(PFBS_ERR_NOMEM, "hipHostMalloc", e);
    }
    return PFBS_OK;
}

pfbs_status pfbs_host_free(void *p) {
    if (!p) return PFBS_OK;
    hipError_t e = hipHostFree(p);
    return e == hipSuccess ? PFBS_OK : err(PFBS_ERR_DEVICE, "hipHostFree", e);
}

pfbs_status pfbs_hstream_create(pfbs_hstream **out, const pfbs_plan_desc *desc, int64_t max_block_samples,
                                int32_t depth) {
    if (!out) return err(PFBS_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (!desc) return err(PFBS_ERR_INVALID, "desc is NULL");
    if (depth < 2 || depth > 16) return err(PFBS_ERR_INVALID, "depth must be 2..16");
    if (max_block_samples <= 0 || desc->N <= 0 || max_block_samples % desc->N != 0)
        return err(PFBS_ERR_INVALID, "max_block_samples must be a positive multiple of N");
    pfbs_hstream *s = new (std::nothrow) pfbs_hstream();
    if (!s) return err(PFBS_ERR_NOMEM, "host allocation");
    s->magic = kLive;
    s->device = -1;
    pfbs_status st = pfbs_plan_create_ex(&s->plan, desc);
    if (st != PFBS_OK) {
        delete s;
        return st;  // the plan recorded its own error text
    }
    pfbs_plan_get_info(s->plan, &s->info);
    hipError_t e = hipGetDevice(&s->device);
    s->max_block = max_block_samples;
    s->depth = depth;
    // a block of B samples completes at most B/(N n_int) + 1 dumps
    s->slot_cap = max_block_samples / s->info.N / s->info.n_int + 1;
    const size_t blk_bytes = (size_t)max_block_samples * 2 * s->info.n_pol;
    const size_t dump_bytes = (size_t)s->slot_cap * s->info.n_prod * s->info.N * sizeof(float);
    s->d_blk.assign(depth, nullptr);
    s->d_dumps.assign(depth, nullptr);
    s->ev_in.assign(depth, nullptr);
    s->ev_comp.assign(depth, nullptr);
    s->ev_out.assign(depth, nullptr);
    s->used.assign(depth, false);
    for (int k = 0; k < depth && e == hipSuccess; ++k) {
        if ((e = hipMalloc(&s->d_blk[k], blk_bytes)) != hipSuccess) break;
        if ((e = hipMalloc((void **)&s->d_dumps[k], dump_bytes)) != hipSuccess) break;
        if ((e = hipEventCreateWithFlags(&s->ev_in[k], hipEventDisableTiming)) != hipSuccess) break;
        if ((e = hipEventCreateWithFlags(&s->ev_comp[k], hipEventDisableTiming)) != hipSuccess) break;
        e = hipEventCreateWithFlags(&s->ev_out[k], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->s_in, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->s_comp, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->s_out, hipStreamNonBlocking);
    if (e != hipSuccess) {
        release(s);
        delete s;
        return err(e == hipErrorOutOfMemory ? PFBS_ERR_NOMEM : PFBS_ERR_DEVICE, "host stream resources", e);
    }
    *out = s;
    return PFBS_OK;
}

pfbs_status pfbs_hstream_push(pfbs_hstream *s, const void *h_block, int64_t n_time_samples, float *h_dumps,
                              int64_t dump_capacity, int64_t *n_dumps_written) {
    if (!s || s->magic != kLive) return err(PFBS_ERR_STATE, "not a live host stream");
    if (!n_dumps_written) return err(PFBS_ERR_INVALID, "n_dumps_written is NULL");
    if (!h_block) return err(PFBS_ERR_INVALID, "h_block is NULL");
    if (n_time_samples <= 0 || n_time_samples > s->max_block || n_time_samples % s->info.N != 0)
        return err(PFBS_ERR_INVALID, "n_time_samples must be a positive multiple of N, at most max_block_samples");
    const int64_t nd = pfbs_dumps_in(s->plan, n_time_samples);
    if (nd < 0) return err(PFBS_ERR_INVALID, "block size");
    if (dump_capacity < nd) return err(PFBS_ERR_INVALID, "dump_capacity is smaller than the dumps this block completes");
    if (nd > 0 && !h_dumps) return err(PFBS_ERR_INVALID, "h_dumps is NULL but dumps complete");
    hipError_t e = hipSetDevice(s->device);
    if (e != hipSuccess) return err(PFBS_ERR_DEVICE, "hipSetDevice", e);
    const int k = (int)(s->pushes % s->depth);
    if (s->used[k] && (e = hipEventSynchronize(s->ev_out[k])) != hipSuccess)
        return err(PFBS_ERR_DEVICE, "waiting for a free slot", e);
    const size_t bytes = (size_t)n_time_samples * 2 * s->info.n_pol;
    if ((e = hipMemcpyAsync(s->d_blk[k], h_block, bytes, hipMemcpyHostToDevice, s->s_in)) != hipSuccess ||
        (e = hipEventRecord(s->ev_in[k], s->s_in)) != hipSuccess ||
        (e = hipStreamWaitEvent(s->s_comp, s->ev_in[k], 0)) != hipSuccess)
        return err(PFBS_ERR_DEVICE, "block copy", e);
    int64_t got = 0;
    pfbs_status st = pfbs_execute(s->plan, s->d_blk[k], n_time_samples, s->d_dumps[k], s->slot_cap, &got, s->s_comp);
    if (st != PFBS_OK) return st;
    if ((e = hipEventRecord(s->ev_comp[k], s->s_comp)) != hipSuccess ||
        (e = hipStreamWaitEvent(s->s_out, s->ev_comp[k], 0)) != hipSuccess)
        return err(PFBS_ERR_DEVICE, "compute event", e);
    if (got > 0 &&
        (e = hipMemcpyAsync(h_dumps, s->d_dumps[k], (size_t)got * s->info.n_prod * s->info.N * sizeof(float),
                            hipMemcpyDeviceToHost, s->s_out)) != hipSuccess)
        return err(PFBS_ERR_DEVICE, "dump copy", e);
    if ((e = hipEventRecord(s->ev_out[k], s->s_out)) != hipSuccess) return err(PFBS_ERR_DEVICE, "copy event", e);
    s->used[k] = true;
    ++s->pushes;
    *n_dumps_written = got;
    return PFBS_OK;
}

pfbs_status pfbs_hstream_sync(pfbs_hstream *s) {
    if (!s || s->magic != kLive) return err(PFBS_ERR_STATE, "not a live host stream");
    hipError_t e = hipSetDevice(s->device);
    if (e == hipSuccess) e = hipStreamSynchronize(s->s_in);
    if (e == hipSuccess) e = hipStreamSynchronize(s->s_comp);
    if (e == hipSuccess) e = hipStreamSynchronize(s->s_out);
    return e == hipSuccess ? PFBS_OK : err(PFBS_ERR_DEVICE, "synchronise", e);
}

pfbs_status pfbs_hstream_destroy(pfbs_hstream *s) {
    if (!s) return PFBS_OK;
    if (s->magic != kLive) return err(PFBS_ERR_STATE, "not a live host stream");
    release(s);
    s->magic = 0;
    delete s;
    return PFBS_OK;
}

pfbs_plan *pfbs_hstream_plan(pfbs_hstream *s) {
    return (s && s->magic == kLive) ? s->plan : nullptr;
}

}  // extern "C"
