// Serving runtime of librotseq: resident matrices swept repeatedly, with
// sweeps of different matrices batched into one preparation launch per
// stage and one chain sweep launch (the batch path), by one worker thread.
// The C ABI is declared in include/rotseq.h.
//
// Life of a sweep: submit copies C and S into pinned host memory and queues
// the sweep behind earlier work on its matrix.  The worker admits pending
// matrices while the device budget allows, takes the head of every resident
// matrix's queue (one sweep per matrix at a time: sweeps of one matrix are
// sequential), copies the batch's coefficients and item table to a device
// arena on the upload stream and launches the batch on the compute stream
// behind that copy.  Two batches can be in flight, so the copies of one
// overlap the sweep of the other.  Reads and closes travel through the same
// per-matrix queues, so they are ordered with the sweeps.
#include "rotseq.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "rotseq_internal.h"

namespace rotseq {
namespace {

using Clock = std::chrono::steady_clock;

// Pinned host blocks in power-of-two size classes, reused across sweeps.
class PinnedPool {
public:
    void *get(size_t bytes, size_t &cls)
    {
        cls = 256;
        while (cls < bytes)
            cls <<= 1;
        {
            std::lock_guard<std::mutex> lock(mu_);
            auto &v = free_[cls];
            if (!v.empty()) {
                void *p = v.back();
                v.pop_back();
                return p;
            }
        }
        void *p = nullptr;
        if (hipHostMalloc(&p, cls, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        return p;
    }
    void put(void *p, size_t cls)
    {
        if (!p)
            return;
        std::lock_guard<std::mutex> lock(mu_);
        free_[cls].push_back(p);
    }
    ~PinnedPool()
    {
        for (auto &kv : free_)
            for (void *p : kv.second)
                (void)hipHostFree(p);
    }

private:
    std::mutex mu_;
    std::map<size_t, std::vector<void *>> free_;
};

enum class Op { kSweep, kRead, kClose };

struct Task {
    Op op;
    int64_t ticket = 0;
    // sweep
    int64_t k = 0;
    double *cs = nullptr;  // pinned: C then S, each (n-1) x k contiguous
    size_t cs_class = 0;
    double flops = 0.0;
    // read
    double *host = nullptr;
    int64_t host_ld = 0;
    // outcome
    bool done = false;
    int status = 0;
    double submit_us = 0.0, start_us = 0.0, end_us = 0.0;
};

enum class State { kPending, kResident, kFreed };

struct Matrix {
    int64_t id = 0, m = 0, n = 0;
    size_t bytes = 0;
    State state = State::kPending;
    double *init = nullptr;    // pinned host copy until its upload completed
    size_t init_class = 0;
    double *dA = nullptr;      // lda = m (at least 1)
    bool async_alloc = false;  // dA from hipMallocAsync
    std::deque<Task *> queue;
    bool inflight = false;
    bool failed = false;
    bool closed = false;  // close requested: no new submits
};

struct InFlight {
    std::vector<Task *> tasks;
    std::vector<Matrix *> mats;
    hipEvent_t done = nullptr;
    int slot = 0;
};

struct Arena {
    void *dev = nullptr;
    size_t bytes = 0;
    void *table = nullptr;  // pinned item table, then zeroed error words
    size_t table_bytes = 0;
    int *words = nullptr;   // pinned copy of the items' error words after the batch
    size_t words_cap = 0;   // entries
};

}  // namespace
}  // namespace rotseq

struct rotseq_server {
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread worker;
    bool stop = false;
    int device = 0;
    uint64_t budget = 0;
    int max_batch = 512;
    int *status = nullptr;
    size_t max_lds = 0;
    int cus = 0;
    rotseq::Clock::time_point t0;
    int64_t next_id = 1, next_ticket = 1;
    std::map<int64_t, rotseq::Matrix *> mats;
    std::deque<rotseq::Matrix *> admit;  // pending, in open order
    std::map<int64_t, rotseq::Task *> tickets;
    uint64_t resident = 0, peak = 0;
    // statistics
    std::vector<double> lat_us;
    int64_t done = 0, failed = 0, batches = 0, batched_sweeps = 0;
    double flops = 0.0, first_submit_us = -1.0, last_end_us = 0.0;
    // worker-only state
    hipStream_t up = nullptr, comp = nullptr;
    hipEvent_t up_done = nullptr;
    // Pinned admission copies whose upload may still be running.
    std::vector<std::pair<hipEvent_t, rotseq::Matrix *>> uploading;
    rotseq::Arena arena[2];
    rotseq::PinnedPool pinned;
    size_t rr = 0;  // round-robin start over resident matrices
};

namespace rotseq {
namespace {

double now_us(const rotseq_server *s)
{
    return std::chrono::duration<double, std::micro>(Clock::now() - s->t0).count();
}

// Finishes a task (lock held).
void finish(rotseq_server *s, Task *t, int status, double end_us)
{
    t->status = status;
    t->end_us = end_us;
    t->done = true;
    if (t->op == Op::kSweep) {
        if (t->cs) {
            s->pinned.put(t->cs, t->cs_class);
            t->cs = nullptr;
        }
        if (status == 0) {
            s->done += 1;
            s->flops += t->flops;
            s->lat_us.push_back(end_us - t->submit_us);
            s->last_end_us = std::max(s->last_end_us, end_us);
        } else {
            s->failed += 1;
        }
    }
}

// Admits pending matrices in open order while the budget allows (lock held).
// Allocation and upload are ordered on the upload stream, which every later
// batch, read and free waits for, so admission never blocks the worker.
void admit(rotseq_server *s)
{
    while (!s->admit.empty()) {
        Matrix *M = s->admit.front();
        if (s->resident + M->bytes > s->budget)
            break;
        s->admit.pop_front();
        double *d = nullptr;
        int rc = ROTSEQ_SUCCESS;
        if (hipMallocAsync((void **)&d, M->bytes, s->up) == hipSuccess) {
            M->async_alloc = true;
        } else {
            (void)hipGetLastError();
            if (hipMalloc(&d, M->bytes) != hipSuccess) {
                (void)hipGetLastError();
                d = nullptr;
                rc = ROTSEQ_E_NOMEM;
            }
        }
        hipEvent_t ev = nullptr;
        if (!rc && (hipMemcpyAsync(d, M->init, M->bytes, hipMemcpyHostToDevice, s->up) != hipSuccess ||
                    hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess ||
                    hipEventRecord(ev, s->up) != hipSuccess))
            rc = ROTSEQ_E_HIP;
        if (ev)
            s->uploading.emplace_back(ev, M);
        else {
            (void)hipStreamSynchronize(s->up);
            s->pinned.put(M->init, M->init_class);
            M->init = nullptr;
        }
        M->state = State::kResident;
        M->dA = d;
        s->resident += M->bytes;
        s->peak = std::max(s->peak, s->resident);
        if (rc)
            M->failed = true;
    }
}

// Returns the pinned admission copies whose uploads have completed.
void reap_uploads(rotseq_server *s)
{
    auto &v = s->uploading;
    for (size_t i = 0; i < v.size();) {
        if (hipEventQuery(v[i].first) == hipSuccess) {
            s->pinned.put(v[i].second->init, v[i].second->init_class);
            v[i].second->init = nullptr;
            (void)hipEventDestroy(v[i].first);
            v[i] = v.back();
            v.pop_back();
        } else {
            ++i;
        }
    }
}

// Runs queue heads that need no kernel: reads, closes and sweeps of failed
// matrices (lock held; the matrix has nothing in flight).
void run_host_heads(rotseq_server *s, Matrix *M)
{
    while (!M->queue.empty() && !M->inflight) {
        Task *t = M->queue.front();
        if (t->op == Op::kSweep && !M->failed)
            return;
        M->queue.pop_front();
        const double at = now_us(s);
        if (t->op == Op::kSweep) {
            finish(s, t, ROTSEQ_E_FAILED, at);
        } else if (t->op == Op::kRead) {
            // Nothing of this matrix is in flight on the compute stream; the
            // upload stream orders the copy after its admission upload.
            const size_t row = (size_t)M->m * sizeof(double);
            int rc = M->failed ? ROTSEQ_E_FAILED : ROTSEQ_SUCCESS;
            if (!rc && M->m > 0 && M->n > 0 &&
                (hipMemcpy2DAsync(t->host, (size_t)t->host_ld * sizeof(double), M->dA, row, row,
                                  (size_t)M->n, hipMemcpyDeviceToHost, s->up) != hipSuccess ||
                 hipStreamSynchronize(s->up) != hipSuccess))
                rc = ROTSEQ_E_HIP;
            finish(s, t, rc, at);
        } else {
            // Freed behind everything already queued on both streams.
            if (M->dA) {
                (void)hipEventRecord(s->up_done, s->up);
                (void)hipStreamWaitEvent(s->comp, s->up_done, 0);
                if (M->async_alloc)
                    (void)hipFreeAsync(M->dA, s->comp);
                else {
                    (void)hipStreamSynchronize(s->comp);
                    (void)hipFree(M->dA);
                }
            }
            M->dA = nullptr;
            s->resident -= M->bytes;
            M->state = State::kFreed;
            delete t;  // nobody waits for a close
            t = nullptr;
        }
        s->cv_done.notify_all();
    }
}

// Collects up to max_batch sweeps, one per resident matrix (lock held).
void collect(rotseq_server *s, std::vector<Task *> &tasks, std::vector<Matrix *> &mats)
{
    std::vector<Matrix *> res;
    for (auto &kv : s->mats)
        if (kv.second->state == State::kResident)
            res.push_back(kv.second);
    if (res.empty())
        return;
    const size_t start = s->rr % res.size();
    for (size_t i = 0; i < res.size() && (int)tasks.size() < s->max_batch; ++i) {
        Matrix *M = res[(start + i) % res.size()];
        run_host_heads(s, M);
        if (M->inflight || M->queue.empty() || M->state != State::kResident)
            continue;
        Task *t = M->queue.front();
        M->queue.pop_front();
        M->inflight = true;
        tasks.push_back(t);
        mats.push_back(M);
    }
    s->rr = start + 1;
}

// Copies the batch's coefficients and item table into arena `slot` and
// launches it; returns the ROTSEQ_E_* code (worker only, lock not held).
int launch(rotseq_server *s, InFlight &f)
{
    Arena &ar = s->arena[f.slot];
    const int count = (int)f.tasks.size();
    std::vector<BatchEntry> entries(count);
    size_t cs_bytes = 0;
    for (int i = 0; i < count; ++i)
        cs_bytes += 2 * (size_t)(f.mats[i]->n - 1) * f.tasks[i]->k * sizeof(double);
    // The coefficients go first in the arena, then the batch block.
    const size_t cs_region = (cs_bytes + 255) & ~(size_t)255;
    size_t off = 0;
    for (int i = 0; i < count; ++i) {
        Matrix *M = f.mats[i];
        Task *t = f.tasks[i];
        const int64_t n1 = M->n - 1;
        entries[i] = BatchEntry{M->dA, (const void *)off, (const void *)(off + n1 * t->k * sizeof(double)),
                                M->m, M->n, t->k, std::max<int64_t>(1, M->m), n1, n1};
        off += 2 * (size_t)n1 * t->k * sizeof(double);
    }
    std::vector<BatchItem> items;
    BatchLaunch L{};
    const size_t block = batch_layout(entries.data(), count, 8, 8, items, L);
    const size_t need = cs_region + block;
    if (ar.bytes < need) {
        if (ar.dev)
            (void)hipFree(ar.dev);
        ar.dev = nullptr;
        ar.bytes = 0;
        const size_t want = need + need / 2;
        if (hipMalloc(&ar.dev, want) != hipSuccess) {
            (void)hipGetLastError();
            return ROTSEQ_E_NOMEM;
        }
        ar.bytes = want;
    }
    // The item table and the items' zeroed error words are one upload.
    const size_t table = L.status_off + (size_t)count * sizeof(int);
    if (ar.words_cap < (size_t)count) {
        if (ar.words)
            (void)hipHostFree(ar.words);
        ar.words = nullptr;
        ar.words_cap = 0;
        if (hipHostMalloc((void **)&ar.words, (size_t)count * 2 * sizeof(int), hipHostMallocDefault) !=
            hipSuccess) {
            (void)hipGetLastError();
            return ROTSEQ_E_NOMEM;
        }
        ar.words_cap = (size_t)count * 2;
    }
    if (ar.table_bytes < table) {
        if (ar.table)
            (void)hipHostFree(ar.table);
        ar.table = nullptr;
        ar.table_bytes = 0;
        if (hipHostMalloc(&ar.table, table * 2, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return ROTSEQ_E_NOMEM;
        }
        ar.table_bytes = table * 2;
    }
    const uintptr_t base = (uintptr_t)ar.dev;
    for (int i = 0; i < count; ++i) {
        items[i].C = (const void *)(base + (uintptr_t)items[i].C);
        items[i].S = (const void *)(base + (uintptr_t)items[i].S);
    }
    batch_rebase(items, base + cs_region);
    L.arith = kLift;
    L.publish = 1;
    L.spin_limit = wait_spin_limit();
    L.wait_bias = wait_bias();
    L.items = (const BatchItem *)(base + cs_region);
    int waves = 8;
    size_t lds = chain_lds_bytes(8, waves, 8);
    while (waves > 1 && lds > s->max_lds)
        lds = chain_lds_bytes(8, --waves, 8);
    L.waves = waves;
    L.lds_bytes = lds;
    L.nwg = batch_assign_workgroups(items, waves);
    std::memcpy(ar.table, items.data(), items.size() * sizeof(BatchItem));
    std::memset((char *)ar.table + L.status_off, 0, (size_t)count * sizeof(int));
    // Uploads on the upload stream; the previous use of this arena slot has
    // completed (its batch was retired before the slot was reused).
    off = 0;
    for (int i = 0; i < count; ++i) {
        const size_t b = 2 * (size_t)(f.mats[i]->n - 1) * f.tasks[i]->k * sizeof(double);
        if (hipMemcpyAsync((char *)ar.dev + off, f.tasks[i]->cs, b, hipMemcpyHostToDevice, s->up) !=
            hipSuccess)
            return ROTSEQ_E_HIP;
        off += b;
    }
    if (hipMemcpyAsync((void *)L.items, ar.table, table, hipMemcpyHostToDevice, s->up) != hipSuccess)
        return ROTSEQ_E_HIP;
    if (hipEventRecord(s->up_done, s->up) != hipSuccess ||
        hipStreamWaitEvent(s->comp, s->up_done, 0) != hipSuccess)
        return ROTSEQ_E_HIP;
    if (launch_prep_batch(L, s->comp) != hipSuccess || launch_chain_batch(L, s->comp) != hipSuccess)
        return ROTSEQ_E_HIP;
    // The items' error words come back with the batch (read in retire).
    if (hipMemcpyAsync(ar.words, (const char *)L.items + L.status_off, (size_t)count * sizeof(int),
                       hipMemcpyDeviceToHost, s->comp) != hipSuccess)
        return ROTSEQ_E_HIP;
    if (hipEventRecord(f.done, s->comp) != hipSuccess)
        return ROTSEQ_E_HIP;
    return ROTSEQ_SUCCESS;
}

// Finishes the sweeps of a batch: `rc` for all of them if the launch or the
// wait failed, else each sweep's own error word (a bounded wait of its
// kernel that gave up leaves its matrix wrong: ROTSEQ_E_TIMEOUT).  A failed
// sweep fails the later sweeps of its matrix.
void retire(rotseq_server *s, InFlight &f, int rc)
{
    if (rc == ROTSEQ_SUCCESS && hipEventSynchronize(f.done) != hipSuccess)
        rc = ROTSEQ_E_HIP;
    const int *words = rc == ROTSEQ_SUCCESS ? s->arena[f.slot].words : nullptr;
    std::lock_guard<std::mutex> lock(s->mu);
    const double at = now_us(s);
    for (size_t i = 0; i < f.tasks.size(); ++i) {
        int st = rc;
        if (words && words[i] != 0)
            st = ROTSEQ_E_TIMEOUT;
        finish(s, f.tasks[i], st, at);
        f.mats[i]->inflight = false;
        if (st)
            f.mats[i]->failed = true;
        run_host_heads(s, f.mats[i]);
    }
    s->batches += 1;
    s->batched_sweeps += (int64_t)f.tasks.size();
    s->cv_done.notify_all();
}

void worker_main(rotseq_server *s)
{
    (void)hipSetDevice(s->device);
    std::deque<InFlight> inflight;
    hipEvent_t evs[2];
    (void)hipEventCreateWithFlags(&evs[0], hipEventDisableTiming);
    (void)hipEventCreateWithFlags(&evs[1], hipEventDisableTiming);
    int slot = 0;
    for (;;) {
        // Retire whatever has completed, without blocking.
        while (!inflight.empty() && hipEventQuery(inflight.front().done) == hipSuccess) {
            retire(s, inflight.front(), ROTSEQ_SUCCESS);
            inflight.pop_front();
        }
        InFlight f;
        bool quit = false;
        {
            std::unique_lock<std::mutex> lock(s->mu);
            reap_uploads(s);
            admit(s);
            if (inflight.size() < 2)
                collect(s, f.tasks, f.mats);
            if (f.tasks.empty()) {
                if (inflight.empty()) {
                    // Stop once nothing runnable is left: resident queues
                    // are empty and no pending matrix fits.
                    bool busy = !s->admit.empty() && s->resident + s->admit.front()->bytes <= s->budget;
                    for (auto &kv : s->mats)
                        busy = busy || (!kv.second->queue.empty() && kv.second->state == State::kResident);
                    if (s->stop && !busy)
                        quit = true;
                    else
                        s->cv_work.wait_for(lock, std::chrono::milliseconds(20));
                } else if (inflight.size() < 2) {
                    // A batch is running: wake for new work or poll again soon.
                    s->cv_work.wait_for(lock, std::chrono::microseconds(20));
                }
            } else {
                const double at = now_us(s);
                for (Task *t : f.tasks)
                    t->start_us = at;
            }
        }
        if (quit)
            break;
        if (!f.tasks.empty()) {
            f.slot = slot;
            f.done = evs[slot];
            slot ^= 1;
            const int rc = launch(s, f);
            if (rc)
                retire(s, f, rc);
            else
                inflight.push_back(f);
        } else if (inflight.size() >= 2) {
            retire(s, inflight.front(), ROTSEQ_SUCCESS);  // blocks on the oldest
            inflight.pop_front();
        }
    }
    while (!inflight.empty()) {
        retire(s, inflight.front(), ROTSEQ_SUCCESS);
        inflight.pop_front();
    }
    (void)hipStreamSynchronize(s->up);
    {
        std::lock_guard<std::mutex> lock(s->mu);
        reap_uploads(s);
    }
    (void)hipEventDestroy(evs[0]);
    (void)hipEventDestroy(evs[1]);
}

}  // namespace
}  // namespace rotseq

using namespace rotseq;

extern "C" {

int rotseq_server_create(const rotseq_server_config *cfg, rotseq_server **out)
{
    if (out == nullptr)
        return -2;
    *out = nullptr;
    if (cfg && cfg->max_batch < 0)
        return -1;
    rotseq_server *s = new rotseq_server();
    s->budget = cfg && cfg->hbm_budget_bytes ? cfg->hbm_budget_bytes : (uint64_t)64 << 30;
    s->max_batch = cfg && cfg->max_batch ? cfg->max_batch : 512;
    s->t0 = Clock::now();
    int rc = hipGetDevice(&s->device) == hipSuccess ? ROTSEQ_SUCCESS : ROTSEQ_E_HIP;
    if (!rc)
        rc = device_query(&s->cus, &s->max_lds, &s->status);
    if (!rc && (hipStreamCreateWithFlags(&s->up, hipStreamNonBlocking) != hipSuccess ||
                hipStreamCreateWithFlags(&s->comp, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&s->up_done, hipEventDisableTiming) != hipSuccess))
        rc = ROTSEQ_E_HIP;
    if (rc) {
        delete s;
        return rc;
    }
    s->worker = std::thread(worker_main, s);
    *out = s;
    return ROTSEQ_SUCCESS;
}

int rotseq_server_open(rotseq_server *s, int64_t m, int64_t n, const double *A_host, int64_t lda,
                       rotseq_matrix_id *id)
{
    if (s == nullptr)
        return -1;
    if (m < 0)
        return -2;
    if (n < 0)
        return -3;
    if (A_host == nullptr && m > 0 && n > 0)
        return -4;
    if (lda < std::max<int64_t>(1, m))
        return -5;
    if (id == nullptr)
        return -6;
    Matrix *M = new Matrix();
    M->m = m;
    M->n = n;
    M->bytes = (size_t)std::max<int64_t>(1, m) * (size_t)std::max<int64_t>(1, n) * sizeof(double);
    if (M->bytes > s->budget) {
        delete M;
        return ROTSEQ_E_BUDGET;
    }
    M->init = (double *)s->pinned.get(M->bytes, M->init_class);
    if (M->init == nullptr) {
        delete M;
        return ROTSEQ_E_NOMEM;
    }
    std::memset(M->init, 0, M->bytes);
    for (int64_t j = 0; j < n; ++j)
        if (m > 0)
            std::memcpy(M->init + (size_t)j * m, A_host + j * lda, (size_t)m * sizeof(double));
    {
        std::lock_guard<std::mutex> lock(s->mu);
        M->id = s->next_id++;
        s->mats[M->id] = M;
        s->admit.push_back(M);
        *id = M->id;
    }
    s->cv_work.notify_one();
    return ROTSEQ_SUCCESS;
}

int rotseq_server_submit(rotseq_server *s, rotseq_matrix_id id, int64_t k, const double *C,
                         int64_t ldc, const double *S, int64_t lds, rotseq_ticket *ticket)
{
    if (s == nullptr)
        return -1;
    if (k < 0)
        return -3;
    if (ticket == nullptr)
        return -8;
    int64_t m = 0, n = 0;
    {
        std::lock_guard<std::mutex> lock(s->mu);
        auto it = s->mats.find(id);
        if (it == s->mats.end())
            return ROTSEQ_E_INVAL;
        if (it->second->closed)
            return ROTSEQ_E_CLOSED;
        m = it->second->m;
        n = it->second->n;
    }
    const int64_t n1 = std::max<int64_t>(n - 1, 0);
    const bool work = m > 0 && n > 1 && k > 0;
    if (work && C == nullptr)
        return -4;
    if (ldc < std::max<int64_t>(1, n1))
        return -5;
    if (work && S == nullptr)
        return -6;
    if (lds < std::max<int64_t>(1, n1))
        return -7;
    Task *t = new Task();
    t->op = Op::kSweep;
    t->k = k;
    t->flops = 6.0 * (double)m * (double)n1 * (double)k;
    if (work) {
        const size_t half = (size_t)n1 * (size_t)k;
        t->cs = (double *)s->pinned.get(2 * half * sizeof(double), t->cs_class);
        if (t->cs == nullptr) {
            delete t;
            return ROTSEQ_E_NOMEM;
        }
        for (int64_t p = 0; p < k; ++p) {
            std::memcpy(t->cs + p * n1, C + p * ldc, (size_t)n1 * sizeof(double));
            std::memcpy(t->cs + half + p * n1, S + p * lds, (size_t)n1 * sizeof(double));
        }
    }
    {
        std::lock_guard<std::mutex> lock(s->mu);
        auto it = s->mats.find(id);
        if (it == s->mats.end() || it->second->closed) {
            if (t->cs)
                s->pinned.put(t->cs, t->cs_class);
            delete t;
            return it == s->mats.end() ? ROTSEQ_E_INVAL : ROTSEQ_E_CLOSED;
        }
        t->ticket = s->next_ticket++;
        t->submit_us = now_us(s);
        if (s->first_submit_us < 0)
            s->first_submit_us = t->submit_us;
        s->tickets[t->ticket] = t;
        if (!work) {
            finish(s, t, ROTSEQ_SUCCESS, t->submit_us);
            t->start_us = t->submit_us;
        } else {
            it->second->queue.push_back(t);
        }
        *ticket = t->ticket;
    }
    s->cv_work.notify_one();
    return ROTSEQ_SUCCESS;
}

int rotseq_server_wait(rotseq_server *s, rotseq_ticket ticket, int64_t timeout_us,
                       rotseq_sweep_info *info)
{
    if (s == nullptr)
        return -1;
    std::unique_lock<std::mutex> lock(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end())
        return ROTSEQ_E_INVAL;
    Task *t = it->second;
    auto ready = [&] { return t->done; };
    if (timeout_us < 0)
        s->cv_done.wait(lock, ready);
    else if (!s->cv_done.wait_for(lock, std::chrono::microseconds(timeout_us), ready))
        return ROTSEQ_E_TIMEOUT;
    if (info) {
        info->status = t->status;
        info->reserved = 0;
        info->submit_us = t->submit_us;
        info->start_us = t->start_us;
        info->end_us = t->end_us;
    }
    return t->status;
}

int rotseq_server_read(rotseq_server *s, rotseq_matrix_id id, double *A_host, int64_t lda)
{
    if (s == nullptr)
        return -1;
    Task *t = new Task();
    {
        std::lock_guard<std::mutex> lock(s->mu);
        auto it = s->mats.find(id);
        if (it == s->mats.end()) {
            delete t;
            return ROTSEQ_E_INVAL;
        }
        Matrix *M = it->second;
        if (M->closed) {
            delete t;
            return ROTSEQ_E_CLOSED;
        }
        if (A_host == nullptr && M->m > 0 && M->n > 0) {
            delete t;
            return -3;
        }
        if (lda < std::max<int64_t>(1, M->m)) {
            delete t;
            return -4;
        }
        t->op = Op::kRead;
        t->host = A_host;
        t->host_ld = lda;
        t->submit_us = now_us(s);
        M->queue.push_back(t);
    }
    s->cv_work.notify_one();
    std::unique_lock<std::mutex> lock(s->mu);
    s->cv_done.wait(lock, [&] { return t->done; });
    const int rc = t->status;
    delete t;
    return rc;
}

int rotseq_server_close(rotseq_server *s, rotseq_matrix_id id)
{
    if (s == nullptr)
        return -1;
    {
        std::lock_guard<std::mutex> lock(s->mu);
        auto it = s->mats.find(id);
        if (it == s->mats.end())
            return ROTSEQ_E_INVAL;
        Matrix *M = it->second;
        if (M->closed)
            return ROTSEQ_E_CLOSED;
        M->closed = true;
        Task *t = new Task();
        t->op = Op::kClose;
        t->submit_us = now_us(s);
        M->queue.push_back(t);
    }
    s->cv_work.notify_one();
    return ROTSEQ_SUCCESS;
}

int rotseq_server_stats_get(rotseq_server *s, rotseq_server_stats *out)
{
    if (s == nullptr)
        return -1;
    if (out == nullptr)
        return -2;
    std::lock_guard<std::mutex> lock(s->mu);
    *out = rotseq_server_stats{};
    out->sweeps_done = s->done;
    out->sweeps_failed = s->failed;
    out->batches = s->batches;
    for (auto &kv : s->mats) {
        out->matrices_resident += kv.second->state == State::kResident;
        out->matrices_pending += kv.second->state == State::kPending;
    }
    out->resident_bytes = s->resident;
    out->peak_resident_bytes = s->peak;
    out->flops = s->flops;
    out->busy_s = s->first_submit_us >= 0 ? (s->last_end_us - s->first_submit_us) * 1e-6 : 0.0;
    out->gflops = out->busy_s > 0 ? s->flops / out->busy_s / 1e9 : 0.0;
    if (!s->lat_us.empty()) {
        std::vector<double> v = s->lat_us;
        auto pct = [&](double q) {
            const size_t i = std::min(v.size() - 1, (size_t)(q * (double)(v.size() - 1) + 0.5));
            std::nth_element(v.begin(), v.begin() + i, v.end());
            return v[i];
        };
        out->p50_us = pct(0.50);
        out->p99_us = pct(0.99);
    }
    out->mean_batch = s->batches ? (double)s->batched_sweeps / (double)s->batches : 0.0;
    return ROTSEQ_SUCCESS;
}

int rotseq_server_destroy(rotseq_server *s)
{
    if (s == nullptr)
        return ROTSEQ_SUCCESS;
    {
        std::lock_guard<std::mutex> lock(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable())
        s->worker.join();
    int rc = hipDeviceSynchronize() == hipSuccess ? ROTSEQ_SUCCESS : ROTSEQ_E_HIP;
    for (auto &kv : s->mats) {
        Matrix *M = kv.second;
        if (M->dA) {
            if (M->async_alloc)
                (void)hipFreeAsync(M->dA, s->comp);
            else
                (void)hipFree(M->dA);
        }
        if (M->init)
            s->pinned.put(M->init, M->init_class);
        // Left only on matrices that were never admitted.  Sweeps are owned
        // by the ticket table; a read would still have a waiting caller,
        // which destroying the server under it does not allow.
        for (Task *t : M->queue)
            if (t->op == Op::kClose)
                delete t;
        delete M;
    }
    for (auto &kv : s->tickets) {
        if (kv.second->cs)
            s->pinned.put(kv.second->cs, kv.second->cs_class);
        delete kv.second;
    }
    for (Arena &a : s->arena) {
        if (a.dev)
            (void)hipFree(a.dev);
        if (a.table)
            (void)hipHostFree(a.table);
        if (a.words)
            (void)hipHostFree(a.words);
    }
    if (s->comp)
        (void)hipStreamSynchronize(s->comp);
    if (s->up)
        (void)hipStreamDestroy(s->up);
    if (s->comp)
        (void)hipStreamDestroy(s->comp);
    if (s->up_done)
        (void)hipEventDestroy(s->up_done);
    delete s;
    return rc;
}

}  // extern "C"
