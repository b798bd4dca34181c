// Sort server: a request loop with continuous batching on one GPU.
//
// Jobs arrive with host data.  A scheduler thread keeps up to `slots` launches
// in flight, each on its own stream with its own pinned staging buffers.
// Whenever a slot is free it admits, in FIFO order, the waiting jobs whose
// device buffers (characters, descriptors, outputs, workspace) fit together into
// the resident HBM arena (the memory budget), packs them into one flat string
// space and enqueues copy-in, one batched sort (one launch sequence over one
// device work queue), and copy-out.  Jobs that arrive while other launches run
// join the next free slot, so their work overlaps on the device.  Completion is
// detected with events; results are copied to the caller's host buffers and the
// arena block is released, which admits the next waiting jobs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <functional>
#include <cstring>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "ssort.h"
#include "ssort_admission.h"

namespace {

using clk = std::chrono::steady_clock;

struct JobRec {
    ssort_job job;
    uint64_t ticket;
    clk::time_point t_submit, t_start, t_done;
    int state = 0;          // 0 waiting, 1 running, 2 done, 3 cancelled
    ssort_status status = SSORT_OK;
    uint64_t device_error = 0;   // the launch's device error mask
};

struct LaunchSlot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    ssort_ctx *ctx = nullptr;
    uint8_t *stage_in = nullptr;    // pinned: chars, starts, lengths, set_begin
    uint32_t *stage_out = nullptr;  // pinned: perm, lcp
    bool busy = false;
    size_t arena_off = 0;
    std::vector<uint64_t> jobs;
    std::vector<uint32_t> set_begin;
};

size_t a256(size_t x) { return (x + 255) / 256 * 256; }

// Small persistent pool for the host-side copies into pinned staging.
class CopyPool {
  public:
    explicit CopyPool(int n) {
        for (int i = 0; i < n; ++i) th_.emplace_back([this] { work(); });
    }
    ~CopyPool() {
        {
            std::lock_guard<std::mutex> lk(m_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto &t : th_) t.join();
    }
    // run f(0..count-1) on the pool and the calling thread; returns when done
    void run(size_t count, const std::function<void(size_t)> &f) {
        if (count == 0) return;
        {
            std::lock_guard<std::mutex> lk(m_);
            f_ = &f;
            count_ = count;
            next_ = 0;
            left_ = count;
            ++gen_;
        }
        cv_.notify_all();
        drain();
        std::unique_lock<std::mutex> lk(m_);
        done_.wait(lk, [&] { return left_ == 0; });
        f_ = nullptr;
    }

  private:
    void drain() {
        for (;;) {
            size_t i;
            const std::function<void(size_t)> *f;
            {
                std::lock_guard<std::mutex> lk(m_);
                if (!f_ || next_ >= count_) return;
                i = next_++;
                f = f_;
            }
            (*f)(i);
            std::lock_guard<std::mutex> lk(m_);
            if (--left_ == 0) done_.notify_all();
        }
    }
    void work() {
        uint64_t seen = 0;
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(m_);
                cv_.wait(lk, [&] { return stop_ || (gen_ != seen && f_ && next_ < count_); });
                if (stop_) return;
                seen = gen_;
            }
            drain();
        }
    }
    std::vector<std::thread> th_;
    std::mutex m_;
    std::condition_variable cv_, done_;
    const std::function<void(size_t)> *f_ = nullptr;
    size_t count_ = 0, next_ = 0, left_ = 0;
    uint64_t gen_ = 0;
    bool stop_ = false;
};

uint64_t job_raw_entries(const ssort_job &j) { return (j.flags & SSORT_TO_END) ? j.n : (uint64_t)j.n + 1; }

struct PackLayout {
    size_t chars, raw, jobs, starts, lengths, setb, perm, lcp, ws, total, stage_in, out_bytes;
    uint64_t nchars, n;
    uint32_t m;
};

uint64_t job_nchars(const ssort_job &j) {
    if (j.flags & SSORT_TO_END) return j.nchars;
    return j.n ? j.offsets[j.n] - j.offsets[0] : 0;
}

}  // namespace

struct ssort_server {
    int device = 0;
    size_t budget = 0, stage_bytes = 0;
    uint32_t max_jobs = 0;
    uint64_t max_strings = 0;
    uint8_t *arena = nullptr;
    ssd::Admission *adm = nullptr;
    CopyPool *pool = nullptr;
    std::vector<LaunchSlot> slots;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::map<uint64_t, JobRec> jobs;
    uint64_t next_ticket = 1;
    std::atomic<bool> stop{false};
    std::thread sched;
    ssort_server_stats_t st{};
    ssort_tuning tun{};

    // Packed device layout of a batch: characters, starts, lengths, set
    // boundaries (copied in as one block), then perm and lcp (copied out as
    // one block), then the sort's workspace.
    PackLayout sizes(uint64_t nchars, uint64_t n, uint32_t m) {
        PackLayout L{};
        L.nchars = nchars;
        L.n = n;
        L.m = m;
        size_t ws = 0;
        ssort_workspace_bytes(slots[0].ctx, (uint32_t)n, m ? m : 1, &ws);
        size_t off = 0;
        // copied in: characters, raw offsets, job table, set boundaries
        L.chars = off; off = a256(off + nchars + 8);
        L.raw = off; off = a256(off + 8 * (n + m));
        L.jobs = off; off = a256(off + sizeof(ssd::PackJob) * m);
        L.setb = off; off = a256(off + 4 * (m + 1));
        L.stage_in = off;
        // built on the device
        L.starts = off; off = a256(off + 8 * n);
        L.lengths = off; off = a256(off + 4 * n);
        // copied out
        L.perm = off; off = a256(off + 4 * n);
        L.lcp = off; off = a256(off + 4 * n);
        L.out_bytes = off - L.perm;
        L.ws = off; off = a256(off + ws);
        L.total = off;
        return L;
    }
    PackLayout layout(const std::vector<uint64_t> &ts) {
        uint64_t nc = 0, n = 0;
        for (uint64_t t : ts) {
            nc += job_nchars(jobs[t].job);
            n += jobs[t].job.n;
        }
        return sizes(nc, n, (uint32_t)ts.size());
    }

    // Launch the admitted jobs on slot s (called with mu held): pack their
    // characters and raw offsets into the slot's pinned staging (copy pool),
    // copy in, build start/length descriptors on the device, sort the batch,
    // copy the permutations and LCP arrays out, record the completion event.
    void launch(LaunchSlot &s, const std::vector<uint64_t> &ts, const PackLayout &L) {
        uint8_t *dev = arena + s.arena_off;
        uint8_t *in = s.stage_in;
        uint64_t *raw = (uint64_t *)(in + L.raw);
        ssd::PackJob *jt = (ssd::PackJob *)(in + L.jobs);
        uint32_t *setb = (uint32_t *)(in + L.setb);
        uint64_t cbase = 0, sbase = 0, rbase = 0;
        s.set_begin.assign(L.m + 1, 0);
        struct Piece { const void *src; void *dst; size_t len; };
        std::vector<Piece> pieces;
        const size_t PIECE = (size_t)8 << 20;
        auto add = [&](const void *src, void *dst, size_t len) {
            for (size_t o = 0; o < len; o += PIECE)
                pieces.push_back({(const uint8_t *)src + o, (uint8_t *)dst + o, std::min(PIECE, len - o)});
        };
        for (uint32_t k = 0; k < L.m; ++k) {
            JobRec &r = jobs[ts[k]];
            const ssort_job &j = r.job;
            r.state = 1;
            r.t_start = clk::now();
            const uint64_t nc = job_nchars(j);
            const uint64_t o0 = (j.flags & SSORT_TO_END) ? 0 : (j.n ? j.offsets[0] : 0);
            add(j.chars + o0, in + L.chars + cbase, nc);
            const uint64_t re = j.n ? job_raw_entries(j) : 0;
            add(j.offsets, raw + rbase, 8 * re);
            jt[k] = ssd::PackJob{cbase, rbase, o0, j.nchars, j.n, j.flags};
            setb[k] = (uint32_t)sbase;
            s.set_begin[k] = (uint32_t)sbase;
            cbase += nc;
            sbase += j.n;
            rbase += re;
        }
        setb[L.m] = (uint32_t)sbase;
        s.set_begin[L.m] = (uint32_t)sbase;
        s.jobs = ts;
        unlocked([&] { pool->run(pieces.size(), [&](size_t i) { memcpy(pieces[i].dst, pieces[i].src, pieces[i].len); }); });
        hipError_t ce = hipMemcpyAsync(dev, in, L.stage_in, hipMemcpyHostToDevice, s.stream);
        if (ce == hipSuccess && L.n) {
            const uint32_t grid = (uint32_t)std::min<uint64_t>((L.n + ssd::NT - 1) / ssd::NT, 4096);
            hipLaunchKernelGGL(ssd::k_pack, dim3(grid), dim3(ssd::NT), 0, s.stream, (const ssd::PackJob *)(dev + L.jobs),
                               (const uint32_t *)(dev + L.setb), L.m, (const unsigned long long *)(dev + L.raw),
                               (unsigned long long *)(dev + L.starts), (uint32_t *)(dev + L.lengths), (uint32_t)L.n);
            ce = hipGetLastError();
        }
        ssort_strings flat{dev + L.chars, L.nchars, (const uint64_t *)(dev + L.starts),
                           (const uint32_t *)(dev + L.lengths), (uint32_t)L.n, 0};
        ssort_status rc = ce == hipSuccess ? ssort_sort_batched(s.ctx, &flat, (const uint32_t *)(dev + L.setb), L.m,
                                                                (uint32_t *)(dev + L.perm), (uint32_t *)(dev + L.lcp),
                                                                dev + L.ws, L.total - L.ws, s.stream)
                                           : SSORT_EDEVICE;
        if (ce == hipSuccess) ce = hipMemcpyAsync(s.stage_out, dev + L.perm, L.out_bytes, hipMemcpyDeviceToHost, s.stream);
        if (ce == hipSuccess) ce = hipEventRecord(s.done, s.stream);
        if (ce != hipSuccess && rc == SSORT_OK) rc = SSORT_EDEVICE;
        s.busy = true;
        st.launches++;
        st.jobs_launched += L.m;
        if (L.m > st.max_jobs_per_launch) st.max_jobs_per_launch = L.m;
        if (rc != SSORT_OK)
            for (uint64_t t : ts) jobs[t].status = rc;
    }

    // The scheduler holds mu except while it copies between the callers'
    // buffers and pinned staging: then submissions and waits go on.  The
    // copies touch only the batch's own buffers (its jobs are running, so no
    // call erases or changes them) and the slot's staging.
    std::unique_lock<std::mutex> *held = nullptr;
    template <typename F>
    void unlocked(F f) {
        if (held) held->unlock();
        f();
        if (held) held->lock();
    }

    void complete(LaunchSlot &s, const PackLayout &L) {
        ssort_status dev_rc = ssort_query_error(s.ctx, s.stream);
        uint64_t bits = 0;
        if (dev_rc != SSORT_OK) {
            ssort_stats_t sst;
            if (ssort_stats(s.ctx, &sst, s.stream) == SSORT_OK) bits = sst.error_bits;
        }
        const uint32_t *perm = s.stage_out;
        const uint32_t *lcp = (const uint32_t *)((const uint8_t *)s.stage_out + (L.lcp - L.perm));
        struct Out { uint32_t *perm, *lcp; uint32_t b, n; };
        std::vector<Out> outs(s.jobs.size());
        for (size_t k = 0; k < s.jobs.size(); ++k) {
            const JobRec &r = jobs.at(s.jobs[k]);
            outs[k] = Out{r.job.out_perm, r.job.out_lcp, s.set_begin[k], r.job.n};
        }
        unlocked([&] {
            pool->run(outs.size(), [&](size_t k) {
                const Out &o = outs[k];
                if (o.perm) memcpy(o.perm, perm + o.b, 4ull * o.n);
                if (o.lcp) memcpy(o.lcp, lcp + o.b, 4ull * o.n);
            });
        });
        const auto now = clk::now();
        for (uint32_t k = 0; k < s.jobs.size(); ++k) {
            JobRec &r = jobs[s.jobs[k]];
            if (r.status == SSORT_OK) r.status = dev_rc;
            r.device_error = bits;
            r.state = 2;
            r.t_done = now;
            st.completed++;
        }
        adm->release(s.arena_off);
        s.busy = false;
        s.jobs.clear();
    }

    void loop() {
        std::vector<PackLayout> lay(slots.size());
        std::unique_lock<std::mutex> lk(mu);
        held = &lk;
        while (!stop) {
            bool progress = false;
            for (size_t i = 0; i < slots.size(); ++i) {
                LaunchSlot &s = slots[i];
                if (s.busy && hipEventQuery(s.done) == hipSuccess) {
                    complete(s, lay[i]);
                    progress = true;
                }
            }
            for (size_t i = 0; i < slots.size(); ++i) {
                LaunchSlot &s = slots[i];
                if (s.busy || adm->waiting() == 0) continue;
                // FIFO prefix whose packed batch fits the arena, the staging
                // buffers and the per-launch limits
                std::vector<uint64_t> ts;
                PackLayout L{};
                uint64_t a_nc = 0, a_n = 0, a_m = 0;
                bool ok = adm->admit_batch(
                    max_jobs,
                    [&](uint64_t t) {
                        const ssort_job &j = jobs[t].job;
                        a_nc += job_nchars(j);
                        a_n += j.n;
                        a_m += 1;
                    },
                    [&]() -> size_t {
                        const PackLayout c = sizes(a_nc, a_n, (uint32_t)a_m);
                        if (c.n > max_strings || c.stage_in > stage_bytes || c.out_bytes > stage_bytes)
                            return (size_t)-1;
                        return c.total;
                    },
                    &ts, &s.arena_off);
                if (!ok || ts.empty()) break;
                L = layout(ts);
                lay[i] = L;
                launch(s, ts, L);
                progress = true;
            }
            if (progress) {
                cv_done.notify_all();
                continue;
            }
            bool any_busy = false;
            for (auto &s : slots) any_busy |= s.busy;
            cv_work.wait_for(lk, std::chrono::microseconds(any_busy ? 20 : 2000));
        }
    }
};

extern "C" {

ssort_status ssort_server_create(int device, size_t hbm_budget, uint32_t slots, const ssort_tuning *t,
                                 const ssort_server_config *cfg, ssort_server **out) {
    if (!out || slots == 0 || slots > 16 || hbm_budget < (1u << 20)) return SSORT_EINVAL;
    *out = nullptr;
    if (hipSetDevice(device) != hipSuccess) return SSORT_EDEVICE;
    ssort_server *S = new ssort_server();
    S->device = device;
    S->budget = hbm_budget;
    S->stage_bytes = cfg && cfg->stage_bytes ? cfg->stage_bytes : (size_t)256 << 20;
    S->max_jobs = cfg && cfg->max_jobs_per_launch ? cfg->max_jobs_per_launch : 4096;
    S->max_strings = cfg && cfg->max_strings_per_launch ? cfg->max_strings_per_launch : (uint64_t)1 << 26;
    if (t) S->tun = *t;
    if (hipMalloc((void **)&S->arena, hbm_budget) != hipSuccess) {
        delete S;
        return SSORT_ENOMEM;
    }
    S->adm = new ssd::Admission(hbm_budget, 256);
    // host copies into and out of pinned staging bound the served throughput:
    // 14 helpers plus the scheduler thread fill a 16-core host share
    S->pool = new CopyPool(14);
    S->slots.resize(slots);
    for (auto &s : S->slots) {
        if (ssort_create(device, t, &s.ctx) != SSORT_OK || hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc((void **)&s.stage_in, S->stage_bytes, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void **)&s.stage_out, S->stage_bytes, hipHostMallocDefault) != hipSuccess) {
            ssort_server_destroy(S);
            return SSORT_ENOMEM;
        }
    }
    S->sched = std::thread([S] { S->loop(); });
    *out = S;
    return SSORT_OK;
}

ssort_status ssort_server_submit(ssort_server *S, const ssort_job *job, uint64_t *ticket) {
    if (!S || !job || !ticket || !job->offsets || (job->n && !job->chars) || !job->out_perm) return SSORT_EINVAL;
    if (job->flags & ~SSORT_TO_END) return SSORT_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    const uint64_t t = S->next_ticket++;
    JobRec &r = S->jobs[t];
    r.job = *job;
    r.ticket = t;
    r.t_submit = clk::now();
    const PackLayout L = S->layout({t});
    if (L.stage_in > S->stage_bytes || L.out_bytes > S->stage_bytes || job->n > S->max_strings ||
        !S->adm->submit(t, L.total)) {
        S->jobs.erase(t);
        return SSORT_EBUSY;
    }
    S->st.submitted++;
    *ticket = t;
    S->cv_work.notify_one();
    return SSORT_OK;
}

ssort_status ssort_server_wait(ssort_server *S, uint64_t ticket, int timeout_ms, ssort_result *res) {
    if (!S) return SSORT_EINVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->jobs.find(ticket);
    if (it == S->jobs.end()) return SSORT_ENOTFOUND;
    auto pred = [&] { return it->second.state >= 2; };
    if (timeout_ms < 0) S->cv_done.wait(lk, pred);
    else if (!S->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), pred)) return SSORT_ETIMEOUT;
    JobRec &r = it->second;
    if (res) {
        res->ticket = ticket;
        res->status = r.status;
        res->latency_ms = std::chrono::duration<double, std::milli>(r.t_done - r.t_submit).count();
        res->queue_ms = r.state == 2 ? std::chrono::duration<double, std::milli>(r.t_start - r.t_submit).count() : 0.0;
        res->device_error = r.device_error;
    }
    const ssort_status rc = r.state == 3 ? SSORT_ENOTFOUND : r.status;
    S->jobs.erase(it);
    return rc;
}

ssort_status ssort_server_cancel(ssort_server *S, uint64_t ticket) {
    if (!S) return SSORT_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->jobs.find(ticket);
    if (it == S->jobs.end() || it->second.state != 0) return SSORT_ENOTFOUND;
    if (!S->adm->cancel(ticket)) return SSORT_ENOTFOUND;
    it->second.state = 3;
    S->cv_done.notify_all();
    return SSORT_OK;
}

ssort_status ssort_server_stats(ssort_server *S, ssort_server_stats_t *out) {
    if (!S || !out) return SSORT_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->st;
    out->arena_used = S->adm->used();
    out->waiting = S->adm->waiting();
    return SSORT_OK;
}

void ssort_server_destroy(ssort_server *S) {
    if (!S) return;
    S->stop = true;
    S->cv_work.notify_all();
    if (S->sched.joinable()) S->sched.join();
    for (auto &s : S->slots) {
        if (s.stream) (void)hipStreamSynchronize(s.stream);
        if (s.stage_in) (void)hipHostFree(s.stage_in);
        if (s.stage_out) (void)hipHostFree(s.stage_out);
        if (s.done) (void)hipEventDestroy(s.done);
        if (s.stream) (void)hipStreamDestroy(s.stream);
        if (s.ctx) ssort_destroy(s.ctx);
    }
    if (S->arena) (void)hipFree(S->arena);
    delete S->adm;
    delete S->pool;
    delete S;
}

}  // extern "C"
