// Served form: a request loop that labels frames as they arrive.
//
// Frames are device-resident; submitting one only enqueues a descriptor.  A
// scheduler thread
//   1. admits waiting frames in arrival order while a label slot is free
//      (the slot pool is carved out of the HBM budget given at creation),
//   2. hands admitted frames to every idle worker -- each worker owns a HIP
//      stream, a batch context and its graph -- as one batch of up
//      to max_batch frames (continuous batching: frames that arrive while
//      other batches run are admitted and launched on the next free worker,
//      so their work overlaps on the device),
//   3. polls the workers' completion events and stamps every finished frame.
// In plain mode (one worker, max_batch 1) each frame is one ccl_label_2d
// call, which is the per-frame baseline the batched mode is compared with.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "ccl.h"
#include "ccl_internal.h"

using namespace ccl;

namespace {

using Clock = std::chrono::steady_clock;

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now().time_since_epoch())
        .count();
}

struct Frame {
    ccl_image_desc d;  // labels filled in at admission (the slot)
    uint64_t tag;
    int64_t t_submit, t_admit, t_launch, t_done;
    int32_t slot;
};

struct Worker {
    hipStream_t stream = nullptr;
    ccl_ctx *ctx = nullptr;
    hipEvent_t done = nullptr;
    std::vector<Frame> batch;
    bool busy = false;
};

}  // namespace

struct ccl_server {
    ccl_server_opts opts{};
    int dev = 0;
    int64_t slot_pixels = 0;
    uint32_t *slot_mem = nullptr;
    int32_t n_slots = 0;
    std::vector<int32_t> free_slots;
    std::vector<uint8_t> held;     // per slot: admitted and not yet released
    std::vector<Worker> workers;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Frame> arrivals;   // submitted, waiting for a slot
    std::deque<Frame> admitted;   // holding a slot, waiting for a worker
    std::deque<Frame> completed;  // finished, waiting to be polled
    int64_t in_flight = 0;        // submitted and not yet completed
    std::atomic<bool> stop{false};
    int error = CCL_OK;
    std::thread thread;
};

namespace {

void run_loop(ccl_server *s) {
    (void)hipSetDevice(s->dev);
    std::vector<ccl_image_desc> descs;
    while (true) {
        bool progressed = false;
        // completions
        for (Worker &w : s->workers) {
            if (!w.busy) continue;
            const hipError_t q = hipEventQuery(w.done);
            if (q == hipErrorNotReady) continue;
            const int64_t t = now_ns();
            std::lock_guard<std::mutex> lk(s->mu);
            if (q != hipSuccess && s->error == CCL_OK) s->error = fail_hip(q);
            for (Frame &f : w.batch) {
                f.t_done = t;
                s->completed.push_back(f);
                --s->in_flight;
            }
            w.batch.clear();
            w.busy = false;
            progressed = true;
        }
        {
            std::unique_lock<std::mutex> lk(s->mu);
            // admission: arrival order, while a slot is free
            while (!s->arrivals.empty() && !s->free_slots.empty()) {
                Frame f = s->arrivals.front();
                s->arrivals.pop_front();
                f.slot = s->free_slots.back();
                s->free_slots.pop_back();
                s->held[(size_t)f.slot] = 1;
                f.d.labels = s->slot_mem + (size_t)f.slot * (size_t)s->slot_pixels;
                f.t_admit = now_ns();
                s->admitted.push_back(f);
                progressed = true;
            }
            if (s->stop.load() && s->in_flight == 0) break;
            // hand batches to idle workers
            for (Worker &w : s->workers) {
                if (w.busy || s->admitted.empty()) continue;
                int64_t px = 0;
                while (!s->admitted.empty() && (int32_t)w.batch.size() < s->opts.max_batch) {
                    const Frame &f = s->admitted.front();
                    const int64_t fp = (int64_t)f.d.H * f.d.W;
                    if (!w.batch.empty() && px + fp > s->opts.max_batch_pixels) break;
                    px += fp;
                    w.batch.push_back(f);
                    s->admitted.pop_front();
                }
                lk.unlock();
                const int64_t t = now_ns();
                int rc;
                if (s->opts.plain) {
                    const Frame &f = w.batch[0];
                    rc = ccl_label_2d(f.d.img, f.d.H, f.d.W, f.d.pitch, s->opts.connectivity,
                                      f.d.labels, w.stream);
                } else {
                    descs.clear();
                    for (const Frame &f : w.batch) descs.push_back(f.d);
                    rc = ccl_label_batch(w.ctx, descs.data(), (int32_t)descs.size(),
                                         s->opts.connectivity, w.stream);
                }
                if (rc == CCL_OK) {
                    const hipError_t e = hipEventRecord(w.done, w.stream);
                    if (e != hipSuccess) rc = fail_hip(e);
                }
                lk.lock();
                for (Frame &f : w.batch) f.t_launch = t;
                if (rc != CCL_OK) {
                    if (s->error == CCL_OK) s->error = rc;
                    for (Frame &f : w.batch) {
                        f.t_done = -1;
                        s->completed.push_back(f);
                        --s->in_flight;
                    }
                    w.batch.clear();
                    continue;
                }
                w.busy = true;
                progressed = true;
            }
            if (!progressed) {
                bool any_busy = false;
                for (const Worker &w : s->workers) any_busy |= w.busy;
                if (any_busy) {
                    // completions are polled: yield the lock briefly
                    lk.unlock();
                    std::this_thread::yield();
                } else {
                    s->cv.wait_for(lk, std::chrono::microseconds(200));
                }
            }
        }
    }
}

void destroy_server(ccl_server *s) {
    for (Worker &w : s->workers) {
        if (w.stream) (void)hipStreamSynchronize(w.stream);
        // plain mode labels through ccl_label_2d, whose workspace is cached
        // per stream: that stream is about to go away
        if (w.stream) release_stream_workspace(w.stream);
        if (w.ctx) (void)ccl_ctx_destroy(w.ctx);
        if (w.done) (void)hipEventDestroy(w.done);
        if (w.stream) (void)hipStreamDestroy(w.stream);
    }
    if (s->slot_mem) (void)hipFree(s->slot_mem);
    delete s;
}

}  // namespace

extern "C" {

int ccl_server_create(ccl_server **out, const ccl_server_opts *o) {
    if (!out || !o) return CCL_ERR_INVALID_ARG;
    *out = nullptr;
    if (o->n_workers < 1 || o->max_batch < 1 || o->max_frame_pixels < 1 ||
        o->max_batch_pixels < o->max_frame_pixels || o->hbm_budget < 1)
        return CCL_ERR_INVALID_ARG;
    if (o->connectivity != 4 && o->connectivity != 8) return CCL_ERR_UNSUPPORTED;
    if (o->plain && (o->n_workers != 1 || o->max_batch != 1)) return CCL_ERR_INVALID_ARG;
    ccl_server *s = new (std::nothrow) ccl_server();
    if (!s) return CCL_ERR_OUT_OF_MEMORY;
    s->opts = *o;
    hipError_t e = hipGetDevice(&s->dev);
    if (e != hipSuccess) {
        delete s;
        return fail_hip(e);
    }
    s->slot_pixels = (int64_t)align_up((size_t)o->max_frame_pixels, 64);
    int64_t n_slots = o->hbm_budget / (s->slot_pixels * (int64_t)sizeof(uint32_t));
    if (n_slots > 0x7FFFFFFF) n_slots = 0x7FFFFFFF;
    if (n_slots < 1) {
        delete s;
        return CCL_ERR_CAPACITY;
    }
    e = hipMalloc(&s->slot_mem, (size_t)n_slots * (size_t)s->slot_pixels * sizeof(uint32_t));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        delete s;
        return CCL_ERR_OUT_OF_MEMORY;
    }
    s->n_slots = (int32_t)n_slots;
    s->held.assign((size_t)n_slots, 0);
    for (int64_t i = n_slots - 1; i >= 0; --i) s->free_slots.push_back((int32_t)i);
    s->workers.resize((size_t)o->n_workers);
    for (Worker &w : s->workers) {
        e = hipStreamCreateWithFlags(&w.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&w.done, hipEventDisableTiming);
        if (e != hipSuccess) {
            destroy_server(s);
            return fail_hip(e);
        }
        if (!o->plain) {
            ccl_ctx_opts co;
            co.max_images = o->max_batch;
            co.max_pixels = o->max_batch_pixels;
            co.cfg = o->cfg;
            co.use_graph = o->use_graph;
            const int rc = ccl_ctx_create(&w.ctx, &co);
            if (rc != CCL_OK) {
                destroy_server(s);
                return rc;
            }
        }
    }
    s->thread = std::thread(run_loop, s);
    *out = s;
    return CCL_OK;
}

int ccl_server_slots(const ccl_server *s, int32_t *n_slots) {
    if (!s || !n_slots) return CCL_ERR_INVALID_ARG;
    *n_slots = s->n_slots;
    return CCL_OK;
}

int ccl_server_submit(ccl_server *s, const uint8_t *img, int32_t H, int32_t W, int64_t pitch,
                      uint64_t tag) {
    if (!s) return CCL_ERR_INVALID_ARG;
    const int rc = validate_image_only(img, H, W, pitch);
    if (rc != CCL_OK) return rc;
    if ((int64_t)H * W > s->opts.max_frame_pixels) return CCL_ERR_CAPACITY;
    Frame f{};
    f.d.img = img;
    f.d.labels = nullptr;
    f.d.H = H;
    f.d.W = W;
    f.d.pitch = pitch;
    f.tag = tag;
    f.t_submit = now_ns();
    f.slot = -1;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop.load()) return CCL_ERR_INVALID_ARG;
        s->arrivals.push_back(f);
        ++s->in_flight;
    }
    s->cv.notify_one();
    return CCL_OK;
}

int ccl_server_poll(ccl_server *s, ccl_frame_result *out, int32_t max, int32_t *n_out) {
    if (!s || !n_out || (max > 0 && !out) || max < 0) return CCL_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    int32_t n = 0;
    while (n < max && !s->completed.empty()) {
        const Frame &f = s->completed.front();
        ccl_frame_result &r = out[n++];
        r.tag = f.tag;
        r.labels = f.d.labels;
        r.slot = f.slot;
        r.t_submit_ns = f.t_submit;
        r.t_admit_ns = f.t_admit;
        r.t_launch_ns = f.t_launch;
        r.t_done_ns = f.t_done;
        s->completed.pop_front();
    }
    *n_out = n;
    return s->error;
}

int ccl_server_release(ccl_server *s, int32_t slot) {
    if (!s || slot < 0) return CCL_ERR_INVALID_ARG;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        // only a slot that an admitted frame holds goes back to the pool: an
        // out-of-range or repeated release would hand one slot to two frames
        if (slot >= s->n_slots || !s->held[(size_t)slot]) return CCL_ERR_INVALID_ARG;
        s->held[(size_t)slot] = 0;
        s->free_slots.push_back(slot);
    }
    s->cv.notify_one();
    return CCL_OK;
}

int ccl_server_pending(ccl_server *s, int64_t *in_flight) {
    if (!s || !in_flight) return CCL_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    *in_flight = s->in_flight;
    return s->error;
}

int ccl_server_destroy(ccl_server *s) {
    if (!s) return CCL_ERR_INVALID_ARG;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop.store(true);
        // frames that never got a slot are dropped (they hold no device memory)
        s->in_flight -= (int64_t)s->arrivals.size();
        s->arrivals.clear();
    }
    s->cv.notify_all();
    // the loop exits once every admitted frame has completed
    if (s->thread.joinable()) s->thread.join();
    const int err = s->error;
    destroy_server(s);
    return err;
}

}  // extern "C"
