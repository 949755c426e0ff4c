// gc_serve.hip - request server: continuous batching of independent coloring
// requests on one GPU (host code only; the kernels are those of the
// single-graph calls).
//
// Threads.  One worker thread per slot.  A worker waits until the oldest
// queued request fits: a slot (itself) is idle and the arena has room for the
// request's footprint.  It then takes the request, copies the graph into its
// arena block on the slot's stream, runs the initial coloring and the
// recoloring passes through the public calls with the slot's context, copies
// the colors back, frees the block and posts a completion record.  Every
// state change (queue, arena, completions) happens under one mutex; GPU work
// happens outside it.
#include "gc_internal.h"
#include "gc_serve.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

namespace {

constexpr int64_t ARENA_ALIGN = 256;

int64_t align_up(int64_t x) { return (x + ARENA_ALIGN - 1) / ARENA_ALIGN * ARENA_ALIGN; }

// First-fit allocator over [0, size): free blocks keyed by offset, merged
// with their neighbors on release.
class Arena {
   public:
    void reset(int64_t size) {
        free_.clear();
        if (size > 0) free_[0] = size;
        size_ = size;
        used_ = peak_ = 0;
    }
    bool alloc(int64_t bytes, int64_t *off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const int64_t rest = it->second - bytes;
            const int64_t at = it->first + bytes;
            free_.erase(it);
            if (rest > 0) free_[at] = rest;
            used_ += bytes;
            peak_ = std::max(peak_, used_);
            return true;
        }
        return false;
    }
    void release(int64_t off, int64_t bytes) {
        auto next = free_.lower_bound(off);
        int64_t start = off, len = bytes;
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                start = prev->first;
                len += prev->second;
                free_.erase(prev);
            }
        }
        if (next != free_.end() && off + bytes == next->first) {
            len += next->second;
            free_.erase(next);
        }
        free_[start] = len;
        used_ -= bytes;
    }
    int64_t size() const { return size_; }
    int64_t used() const { return used_; }
    int64_t peak() const { return peak_; }

   private:
    std::map<int64_t, int64_t> free_;
    int64_t size_ = 0, used_ = 0, peak_ = 0;
};

struct Waiting {
    gc_request req;
    int64_t footprint;
    double t_submit;
};

struct Slot {
    gc_ctx *ctx = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr, evp0 = nullptr, evp1 = nullptr;
};

// Compute-unit mask of slot s out of `slots` on a device of `cus` compute
// units in 8 XCDs: unit i goes to slot (i / (cus / 8) + i) % slots, so every
// slot holds units of every XCD whether the mask's bits count units XCD by
// XCD (i / (cus / 8)) or round robin over the XCDs (i % 8).
std::vector<uint32_t> slot_cu_mask(int cus, int slots, int s, int *count) {
    std::vector<uint32_t> m((size_t)(cus + 31) / 32, 0u);
    const int block = cus / 8 > 0 ? cus / 8 : 1;
    *count = 0;
    for (int i = 0; i < cus; i++)
        if ((i / block + i) % slots == s) {
            m[(size_t)i / 32] |= 1u << (i % 32);
            ++*count;
        }
    return m;
}

int64_t footprint_of(const gc_request &r) {
    return align_up(4 * ((int64_t)r.n + 1)) + align_up(4 * r.nnz) + align_up(4 * (int64_t)r.n);
}

}  // namespace

struct gc_server {
    gc_server_config cfg{};
    char *arena_base = nullptr;
    Arena arena;
    std::mutex mu;
    // Device gate: initial colorings of several slots share the device;
    // a recoloring pass runs alone.  Its persistent walk needs every one of
    // its workgroups resident: kernels of other slots could only delay some of
    // them, but meanwhile the resident ones spin on their dependencies and the
    // device does little else.  Writers (passes) go first once they wait.
    std::mutex gate_mu;
    std::condition_variable gate_cv;
    int gate_shared = 0, gate_waiting = 0;
    bool gate_excl = false;
    bool partitioned = false;  // slots on disjoint compute units: no gate
    int slot_cus = 0;
    hipEvent_t ref = nullptr;  // device time reference of the pass timestamps
    std::condition_variable cv_work, cv_done;
    std::deque<Waiting> queue;
    std::deque<gc_request_done> done;
    std::vector<Slot> slots;
    std::vector<std::thread> workers;
    bool stopping = false;
    int64_t submitted = 0, completed = 0, running = 0, peak_running = 0;
    std::chrono::steady_clock::time_point t0;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    void enter_shared() {
        if (partitioned) return;
        std::unique_lock<std::mutex> lk(gate_mu);
        gate_cv.wait(lk, [&] { return !gate_excl && gate_waiting == 0; });
        gate_shared++;
    }
    void leave_shared() {
        if (partitioned) return;
        std::lock_guard<std::mutex> lk(gate_mu);
        if (--gate_shared == 0) gate_cv.notify_all();
    }
    void enter_excl() {
        if (partitioned) return;
        std::unique_lock<std::mutex> lk(gate_mu);
        gate_waiting++;
        gate_cv.wait(lk, [&] { return !gate_excl && gate_shared == 0; });
        gate_waiting--;
        gate_excl = true;
    }
    void leave_excl() {
        if (partitioned) return;
        std::lock_guard<std::mutex> lk(gate_mu);
        gate_excl = false;
        gate_cv.notify_all();
    }
    void worker(int idx);
    gc_request_done run(int idx, const Waiting &w, int64_t off);
};

gc_request_done gc_server::run(int idx, const Waiting &w, int64_t off) {
    Slot &sl = slots[idx];
    const gc_request &r = w.req;
    gc_request_done d{};
    d.tag = r.tag;
    d.slot = idx;
    d.footprint = w.footprint;
    d.t_submit = w.t_submit;
    char *base = arena_base + off;
    int32_t *rp = (int32_t *)base;
    int32_t *col = (int32_t *)(base + align_up(4 * ((int64_t)r.n + 1)));
    int32_t *colors = (int32_t *)((char *)col + align_up(4 * r.nnz));
    gc_status st = GC_OK;
    auto hip_ok = [&](hipError_t e) {
        if (e != hipSuccess && st == GC_OK) st = GC_ERR_DEVICE;
        return e == hipSuccess;
    };
    hip_ok(hipEventRecord(sl.ev0, sl.stream));
    hip_ok(hipMemcpyAsync(rp, r.row_ptr, 4 * ((size_t)r.n + 1), hipMemcpyHostToDevice, sl.stream));
    if (r.nnz > 0) hip_ok(hipMemcpyAsync(col, r.col_idx, 4 * (size_t)r.nnz, hipMemcpyHostToDevice, sl.stream));
    gc_csr g{r.n, 0, r.nnz, rp, r.nnz > 0 ? col : nullptr};
    gc_stats s0{}, s1{};
    if (st == GC_OK) {
        enter_shared();
        st = gc_init_color(sl.ctx, &g, r.select, r.X, r.seed, 0, 0, colors, &s0, sl.stream);
        hip_ok(hipStreamSynchronize(sl.stream));  // its kernels have left the device
        leave_shared();
    }
    d.rounds = s0.rounds;
    d.colors_init = s0.num_colors;
    d.colors_final = s0.num_colors;
    hip_ok(hipEventRecord(sl.evp0, sl.stream));
    if (partitioned) {
        // the slot's own compute units: the passes go back to back, one synchronization at the end
        for (int32_t p = 0; p < r.passes && st == GC_OK; p++) {
            st = gc_recolor(sl.ctx, &g, r.perm, r.seed, p, colors, colors, p == r.passes - 1 ? &s1 : nullptr,
                            sl.stream);
            if (st == GC_OK && p == r.passes - 1) d.colors_final = s1.num_colors;
        }
    } else {
        for (int32_t p = 0; p < r.passes && st == GC_OK; p++) {
            enter_excl();
            st = gc_recolor(sl.ctx, &g, r.perm, r.seed, p, colors, colors, p == r.passes - 1 ? &s1 : nullptr,
                            sl.stream);
            if (st == GC_OK && p == r.passes - 1) d.colors_final = s1.num_colors;
            hip_ok(hipStreamSynchronize(sl.stream));
            leave_excl();
        }
    }
    hip_ok(hipEventRecord(sl.evp1, sl.stream));
    if (st == GC_OK && r.n > 0)
        hip_ok(hipMemcpyAsync(r.colors, colors, 4 * (size_t)r.n, hipMemcpyDeviceToHost, sl.stream));
    hip_ok(hipEventRecord(sl.ev1, sl.stream));
    hip_ok(hipStreamSynchronize(sl.stream));
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, sl.ev0, sl.ev1) == hipSuccess) d.device_ms = ms;
    if (hipEventElapsedTime(&ms, ref, sl.evp0) == hipSuccess) d.pass_start_ms = ms;
    if (hipEventElapsedTime(&ms, ref, sl.evp1) == hipSuccess) d.pass_end_ms = ms;
    d.status = st;
    return d;
}

void gc_server::worker(int idx) {
    if (hipSetDevice(cfg.device) != hipSuccess) return;
    for (;;) {
        Waiting w{};
        int64_t off = 0;
        {
            std::unique_lock<std::mutex> lk(mu);
            for (;;) {
                if (!queue.empty() && arena.alloc(queue.front().footprint, &off)) break;
                if (stopping && queue.empty()) return;
                cv_work.wait(lk);
            }
            w = queue.front();
            queue.pop_front();
            running++;
            peak_running = std::max(peak_running, running);
        }
        // a request just left the queue: the next one may fit as well
        cv_work.notify_all();
        const double t_admit = now();
        int64_t conc;
        {
            std::lock_guard<std::mutex> lk(mu);
            conc = running;
        }
        gc_request_done d = run(idx, w, off);
        d.t_admit = t_admit;
        d.running_at_admit = (int32_t)conc;
        d.t_done = now();
        {
            std::lock_guard<std::mutex> lk(mu);
            arena.release(off, w.footprint);
            running--;
            completed++;
            done.push_back(d);
        }
        cv_done.notify_all();
        cv_work.notify_all();
    }
}

// Star with `leaves` leaves (center 0) as host CSR.
static void star_csr(int32_t leaves, std::vector<int32_t> &rp, std::vector<int32_t> &col) {
    rp.assign(leaves + 2, 0);
    col.clear();
    for (int32_t i = 1; i <= leaves; i++) col.push_back(i);
    rp[1] = leaves;
    for (int32_t i = 1; i <= leaves; i++) {
        col.push_back(0);
        rp[i + 1] = rp[i] + 1;
    }
}

static gc_status warm_walks(gc_server *s) {
    if (s->cfg.max_n < 65 || s->cfg.max_nnz < 128) return GC_OK;  // slots that cannot hold the warm-up graphs
    int32_t *d = nullptr;
    const size_t ints = 2 * (66 + 128 + 65);
    if (hipMalloc((void **)&d, ints * 4) != hipSuccess) return GC_ERR_OOM;
    gc_status st = GC_OK;
    for (int32_t leaves : {1, 64}) {
        std::vector<int32_t> rp, col;
        star_csr(leaves, rp, col);
        const int32_t n = leaves + 1;
        int32_t *drp = d, *dcol = d + rp.size(), *dc = dcol + col.size();
        if (hipMemcpy(drp, rp.data(), rp.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(dcol, col.data(), col.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
            st = GC_ERR_DEVICE;
            break;
        }
        gc_csr g{n, 0, (int64_t)col.size(), drp, dcol};
        for (Slot &sl : s->slots) {
            gc_stats x{};
            st = gc_init_color(sl.ctx, &g, GC_FIRST_FIT, 1, 1, 0, 0, dc, &x, sl.stream);
            if (st == GC_OK) st = gc_recolor(sl.ctx, &g, GC_PERM_REVERSE, 1, 0, dc, dc, &x, sl.stream);
            if (st != GC_OK) break;
        }
        if (st != GC_OK) break;
    }
    (void)hipFree(d);
    return st;
}

static void server_free(gc_server *s) {
    if (s->ref) (void)hipEventDestroy(s->ref);
    for (Slot &sl : s->slots) {
        if (sl.ev0) (void)hipEventDestroy(sl.ev0);
        if (sl.ev1) (void)hipEventDestroy(sl.ev1);
        if (sl.evp0) (void)hipEventDestroy(sl.evp0);
        if (sl.evp1) (void)hipEventDestroy(sl.evp1);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.ctx) gc_ctx_destroy(sl.ctx);
    }
    if (s->arena_base) (void)hipFree(s->arena_base);
    delete s;
}

extern "C" gc_status gc_server_create(const gc_server_config *cfg, gc_server **out) {
    if (!cfg || !out) return GC_ERR_ARG;
    *out = nullptr;
    if (cfg->slots < 1 || cfg->slots > 64 || cfg->hbm_budget <= 0 || cfg->max_n < 0 || cfg->max_nnz < 0 ||
        cfg->max_n >= INT32_MAX || cfg->max_nnz >= INT32_MAX)
        return GC_ERR_ARG;
    gc_server *s = new (std::nothrow) gc_server();
    if (!s) return GC_ERR_OOM;
    s->cfg = *cfg;
    s->t0 = std::chrono::steady_clock::now();
    if (hipSetDevice(cfg->device) != hipSuccess) {
        delete s;
        return GC_ERR_DEVICE;
    }
    if (hipMalloc((void **)&s->arena_base, (size_t)cfg->hbm_budget) != hipSuccess) {
        s->arena_base = nullptr;
        server_free(s);
        return GC_ERR_OOM;
    }
    s->arena.reset(cfg->hbm_budget);
    s->slots.resize(cfg->slots);
    int dev_cus = 0;
    if (hipDeviceGetAttribute(&dev_cus, hipDeviceAttributeMultiprocessorCount, cfg->device) != hipSuccess) {
        server_free(s);
        return GC_ERR_DEVICE;
    }
    s->slot_cus = dev_cus;
    for (Slot &sl : s->slots) {
        gc_status st = gc_ctx_create(cfg->device, cfg->max_n, cfg->max_nnz, &sl.ctx);
        if (st != GC_OK) {
            sl.ctx = nullptr;
            server_free(s);
            return st;
        }
        if (hipEventCreate(&sl.ev0) != hipSuccess || hipEventCreate(&sl.ev1) != hipSuccess ||
            hipEventCreate(&sl.evp0) != hipSuccess || hipEventCreate(&sl.evp1) != hipSuccess) {
            server_free(s);
            return GC_ERR_DEVICE;
        }
    }
    // compute-unit partitions: at least one unit of every XCD per slot
    s->partitioned = cfg->cu_partition != 0 && dev_cus / cfg->slots >= 8;
    if (s->partitioned) {
        for (int i = 0; i < cfg->slots && s->partitioned; i++) {
            Slot &sl = s->slots[i];
            int cnt = 0;
            std::vector<uint32_t> mask = slot_cu_mask(dev_cus, cfg->slots, i, &cnt);
            if (hipExtStreamCreateWithCUMask(&sl.stream, (uint32_t)mask.size(), mask.data()) != hipSuccess) {
                sl.stream = nullptr;
                (void)hipGetLastError();
                s->partitioned = false;  // the runtime refused the mask: the slots share the device
                break;
            }
            gc_tuning t;
            gc_ctx_get_tuning(sl.ctx, &t);
            t.cu_count = cnt;
            gc_ctx_set_tuning(sl.ctx, &t);
            s->slot_cus = cnt;
        }
        if (!s->partitioned) {
            for (Slot &sl : s->slots) {
                if (sl.stream) (void)hipStreamDestroy(sl.stream);
                sl.stream = nullptr;
                gc_tuning t;
                gc_ctx_get_tuning(sl.ctx, &t);
                t.cu_count = 0;
                gc_ctx_set_tuning(sl.ctx, &t);
            }
            s->slot_cus = dev_cus;
        }
    }
    if (!s->partitioned) {
        for (Slot &sl : s->slots) {
            if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess) {
                sl.stream = nullptr;
                server_free(s);
                return GC_ERR_DEVICE;
            }
        }
    }
    // Size every slot's persistent walk on the idle device (the walk measures
    // how many workgroups are co-resident at its first use): one tiny graph
    // with short rows and one with a row of 64 entries.
    {
        gc_status st = warm_walks(s);
        if (st != GC_OK) {
            server_free(s);
            return st;
        }
    }
    if (hipEventCreate(&s->ref) != hipSuccess || hipEventRecord(s->ref, s->slots[0].stream) != hipSuccess ||
        hipEventSynchronize(s->ref) != hipSuccess) {
        server_free(s);
        return GC_ERR_DEVICE;
    }
    for (int i = 0; i < cfg->slots; i++) s->workers.emplace_back(&gc_server::worker, s, i);
    *out = s;
    return GC_OK;
}

extern "C" gc_status gc_server_submit(gc_server *s, const gc_request *r) {
    if (!s || !r) return GC_ERR_ARG;
    if (r->n < 0 || r->nnz < 0 || r->n > s->cfg.max_n || r->nnz > s->cfg.max_nnz) return GC_ERR_ARG;
    if (!r->row_ptr || (r->nnz > 0 && !r->col_idx) || (r->n > 0 && !r->colors)) return GC_ERR_ARG;
    if (r->select != GC_FIRST_FIT && r->select != GC_RANDOM_X) return GC_ERR_ARG;
    if (r->select == GC_RANDOM_X && (r->X < 1 || r->X > GC_MAX_X)) return GC_ERR_ARG;
    if (r->perm < 0 || r->perm > 3 || r->passes < 0) return GC_ERR_ARG;
    Waiting w{*r, footprint_of(*r), 0.0};
    if (w.footprint > s->arena.size()) return GC_ERR_ARG;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        w.t_submit = s->now();
        s->queue.push_back(w);
        s->submitted++;
    }
    s->cv_work.notify_all();
    return GC_OK;
}

extern "C" gc_status gc_server_poll(gc_server *s, gc_request_done *out, int32_t cap, int32_t *count, int32_t timeout_ms) {
    if (!s || !count || cap < 0 || (cap > 0 && !out)) return GC_ERR_ARG;
    *count = 0;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->done.empty() && timeout_ms != 0) {
        auto ready = [&] { return !s->done.empty(); };
        if (timeout_ms < 0) s->cv_done.wait(lk, ready);
        else s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready);
    }
    int32_t k = 0;
    while (k < cap && !s->done.empty()) {
        out[k++] = s->done.front();
        s->done.pop_front();
    }
    *count = k;
    return GC_OK;
}

extern "C" gc_status gc_server_get_stats(gc_server *s, gc_server_stats *o) {
    if (!s || !o) return GC_ERR_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    o->submitted = s->submitted;
    o->completed = s->completed;
    o->waiting = (int64_t)s->queue.size();
    o->running = s->running;
    o->peak_running = s->peak_running;
    o->arena_size = s->arena.size();
    o->arena_used = s->arena.used();
    o->arena_peak = s->arena.peak();
    o->cu_partition = s->partitioned ? 1 : 0;
    o->slot_cus = s->slot_cus;
    return GC_OK;
}

extern "C" double gc_server_now(gc_server *s) { return s ? s->now() : 0.0; }

extern "C" void gc_server_destroy(gc_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
    }
    s->cv_work.notify_all();
    for (std::thread &t : s->workers) t.join();
    server_free(s);
}
