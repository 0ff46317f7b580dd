// Batch runtime of librotseq: many independent rotation-sequence problems
// (each one Algorithm 2 on its own matrix) prepared by one launch per
// preparation stage and swept by one launch of the chain kernel.  The C ABI
// is declared in include/rotseq.h.
#include "rotseq.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "rotseq_internal.h"

namespace rotseq {

bool resolve_opts(const rotseq_opts *opts, int &arith, int &band, int &kernel);

size_t batch_layout(const BatchEntry *entries, int count, int band, int esize,
                    std::vector<BatchItem> &items, BatchLaunch &L)
{
    constexpr int kUnroll = 16;  // step unroll of the chain kernel
    auto a256 = [](size_t x) { return (x + 255) & ~(size_t)255; };
    items.clear();
    L.status_off = (size_t)count * sizeof(BatchItem);
    size_t off = a256(L.status_off + (size_t)count * sizeof(int));
    int64_t o_neg = 0, o_par = 0, o_sign = 0, o_coef = 0, o_flags = 0, o_all = 0;
    for (int i = 0; i < count; ++i) {
        const BatchEntry &e = entries[i];
        BatchItem it{};
        it.A = e.A;
        it.C = e.C;
        it.S = e.S;
        it.lda = e.lda;
        it.ldc = e.ldc;
        it.lds = e.lds;
        it.m = e.m;
        it.n = e.n;
        it.k = e.k;
        it.npass = (int)((e.k + band - 1) / band);
        it.steps = (int)(((e.n + band - 1 + kUnroll - 1) / kUnroll) * kUnroll);
        it.tiles = (int)((e.m + 63) / 64);
        it.pad = kChainCoefPad;
        const int64_t n1 = e.n - 1;
        it.coef = (void *)off;
        off = a256(off + (size_t)it.npass * (it.steps + it.pad) * band * 2 * esize);
        it.negmask = (uint64_t *)off;
        off = a256(off + (size_t)it.npass * n1 * sizeof(uint64_t));
        it.parity = (uint8_t *)off;
        off = a256(off + (size_t)(it.npass + 1) * n1);
        it.sign = (void *)off;
        off = a256(off + (size_t)e.n * esize);
        it.flags = (int *)off;
        off = a256(off + (size_t)it.tiles * it.npass * sizeof(int));
        it.status = (int *)(L.status_off + (size_t)i * sizeof(int));
        it.off_negmask = o_neg;
        it.off_parity = o_par;
        it.off_sign = o_sign;
        it.off_coef = o_coef;
        it.off_flags = o_flags;
        it.off_all = o_all;
        o_all += std::max<int64_t>(std::max<int64_t>((int64_t)it.npass * (it.steps + it.pad) * band, e.n),
                                   (int64_t)it.tiles * it.npass);
        o_neg += (int64_t)it.npass * n1;
        o_par += n1;
        o_sign += e.n;
        o_coef += (int64_t)it.npass * (it.steps + it.pad) * band;
        o_flags += (int64_t)it.tiles * it.npass;
        items.push_back(it);
    }
    L.count = count;
    L.band = band;
    L.esize = esize;
    L.total_negmask = o_neg;
    L.total_parity = o_par;
    L.total_sign = o_sign;
    L.total_coef = o_coef;
    L.total_flags = o_flags;
    L.total_all = o_all;
    return off;
}

void batch_rebase(std::vector<BatchItem> &items, uintptr_t base)
{
    for (BatchItem &it : items) {
        it.coef = (void *)(base + (uintptr_t)it.coef);
        it.negmask = (uint64_t *)(base + (uintptr_t)it.negmask);
        it.parity = (uint8_t *)(base + (uintptr_t)it.parity);
        it.sign = (void *)(base + (uintptr_t)it.sign);
        it.flags = (int *)(base + (uintptr_t)it.flags);
        it.status = (int *)(base + (uintptr_t)it.status);
    }
}

int64_t batch_assign_workgroups(std::vector<BatchItem> &items, int waves)
{
    int64_t wg = 0;
    for (BatchItem &it : items) {
        it.off_wg = wg;
        const int64_t units = (int64_t)it.tiles * it.npass;
        wg += (units + waves - 1) / waves;
    }
    return wg;
}

namespace {

constexpr int kDefaultWaves = 8;      // waves per workgroup before tuning
constexpr int kTuneWaves[] = {2, 4, 8, 16};

// One entry of the caller's array, type-erased.
struct Entry {
    int64_t m, n, k, lda, ldc, lds;
    void *A;
    const void *C, *S;
};

template <typename P>
Entry entry_of(const P &p)
{
    return Entry{p.m, p.n, p.k, p.lda, p.ldc, p.lds, (void *)p.A, (const void *)p.C, (const void *)p.S};
}

}  // namespace
}  // namespace rotseq

// The plan.  Device memory is one allocation: the item table, then each
// item's workspace (coefficients, lifting signs, progress flags).
struct rotseq_batch {
    int device = 0;
    rotseq::BatchLaunch L{};
    std::vector<rotseq::BatchItem> items;  // host copy, dispatch order
    void *dmem = nullptr;
    size_t dbytes = 0;
    size_t max_lds = 0;
    int cus = 0;
    int64_t waves_total = 0;
    double flops = 0.0, bytes = 0.0;
    int esize = 8;
    std::vector<int64_t> shapes;  // m, n, k of every caller entry, in caller order
    std::vector<int> order;       // caller index of each item (dispatch order)
};

namespace rotseq {
namespace {

int set_waves(rotseq_batch *b, int waves)
{
    const size_t lds = chain_lds_bytes(b->L.band, waves, b->L.esize);
    if (lds > b->max_lds)
        return ROTSEQ_E_UNSUPPORTED;
    int occ = 0;
    if (chain_occupancy(b->L.band, b->L.arith, b->L.esize, waves, lds, &occ, true) != hipSuccess ||
        occ < 1)
        return ROTSEQ_E_UNSUPPORTED;
    const int64_t nwg = batch_assign_workgroups(b->items, waves);
    if (nwg > (int64_t)INT32_MAX)
        return ROTSEQ_E_UNSUPPORTED;
    if (hipMemcpy(b->dmem, b->items.data(), b->items.size() * sizeof(BatchItem),
                  hipMemcpyHostToDevice) != hipSuccess)
        return ROTSEQ_E_HIP;
    b->L.waves = waves;
    b->L.lds_bytes = lds;
    b->L.nwg = nwg;
    return ROTSEQ_SUCCESS;
}

// Entry checks shared by create and update: every entry as rotseq_d checks
// it, then pairwise overlap of the A ranges of the entries with work.
// Returns 0 or -(1000*(idx+1) + argpos); fills `work` with the indices of
// the entries that have work.
int check_entries(int32_t count, const std::vector<Entry> &in, int esize, std::vector<int> &work)
{
    work.clear();
    for (int32_t i = 0; i < count; ++i) {
        const Entry &e = in[i];
        const int bad = check_problem(e.m, e.n, e.k, e.A, e.lda, e.C, e.ldc, e.S, e.lds);
        if (bad)
            return -(1000 * (i + 1) + (-bad));
        if (e.m > 0 && e.n > 1 && e.k > 0)
            work.push_back(i);
    }
    std::vector<std::pair<uintptr_t, int>> starts;
    for (int i : work)
        starts.emplace_back((uintptr_t)in[i].A, i);
    std::sort(starts.begin(), starts.end());
    for (size_t j = 1; j < starts.size(); ++j) {
        const Entry &prev = in[starts[j - 1].second];
        const uintptr_t prev_end =
            starts[j - 1].first + (uintptr_t)esize * (uintptr_t)(prev.lda * (prev.n - 1) + prev.m);
        if (starts[j].first < prev_end)
            return -(1000 * (std::max(starts[j].second, starts[j - 1].second) + 1) + 4);
    }
    return 0;
}

int create(int32_t count, const std::vector<Entry> &in, int esize, const rotseq_opts *opts,
           rotseq_batch **out)
{
    if (out == nullptr)
        return -4;
    *out = nullptr;
    std::vector<int> work;
    const int bad = check_entries(count, in, esize, work);
    if (bad)
        return bad;
    int arith = 0, band = 0, kernel = 0;
    if (!resolve_opts(opts, arith, band, kernel))
        return ROTSEQ_E_UNSUPPORTED;
    if ((kernel != 0 && kernel != kChain) || (opts && (opts->inverse || opts->left)))
        return ROTSEQ_E_UNSUPPORTED;
    if (band == 0)
        band = 8;
    if (band != 4 && band != 6 && band != 8)
        return ROTSEQ_E_UNSUPPORTED;

    rotseq_batch *b = new rotseq_batch();
    if (hipGetDevice(&b->device) != hipSuccess) {
        delete b;
        return ROTSEQ_E_HIP;
    }
    int *status = nullptr;
    int rc = device_query(&b->cus, &b->max_lds, &status);
    if (rc) {
        delete b;
        return rc;
    }
    // Dispatch order: longest sweeps first (a workgroup runs for about
    // `steps` wavefront steps), then longer chains.
    std::sort(work.begin(), work.end(), [&](int x, int y) {
        if (in[x].n != in[y].n)
            return in[x].n > in[y].n;
        if (in[x].k != in[y].k)
            return in[x].k > in[y].k;
        return x < y;
    });
    for (int i : work) {
        if (in[i].n > ((int64_t)1 << 28) || in[i].m > (int64_t)INT32_MAX * 64) {
            delete b;
            return ROTSEQ_E_UNSUPPORTED;
        }
    }
    b->esize = esize;
    for (int32_t i = 0; i < count; ++i) {
        b->shapes.push_back(in[i].m);
        b->shapes.push_back(in[i].n);
        b->shapes.push_back(in[i].k);
    }
    b->order = work;
    std::vector<BatchEntry> ordered;
    for (int i : work) {
        const Entry &e = in[i];
        ordered.push_back(BatchEntry{e.A, e.C, e.S, e.m, e.n, e.k, e.lda, e.ldc, e.lds});
        const int64_t n1 = e.n - 1;
        b->flops += 6.0 * (double)e.m * (double)n1 * (double)e.k;
        b->bytes += (double)esize * (2.0 * (double)e.m * (double)e.n + 2.0 * (double)n1 * (double)e.k);
    }
    const size_t off = batch_layout(ordered.data(), (int)ordered.size(), band, esize, b->items, b->L);
    for (const BatchItem &it : b->items)
        b->waves_total += (int64_t)it.tiles * it.npass;
    b->dbytes = off;
    if (hipMalloc(&b->dmem, b->dbytes) != hipSuccess) {
        (void)hipGetLastError();
        delete b;
        return ROTSEQ_E_NOMEM;
    }
    batch_rebase(b->items, (uintptr_t)b->dmem);
    BatchLaunch &L = b->L;
    L.arith = arith;
    L.publish = 1;
    L.spin_limit = wait_spin_limit();
    L.wait_bias = wait_bias();
    L.items = (const BatchItem *)b->dmem;
    (void)status;
    if (L.count > 0 &&
        hipMemset((char *)b->dmem + L.status_off, 0, (size_t)L.count * sizeof(int)) != hipSuccess) {
        (void)hipFree(b->dmem);
        delete b;
        return ROTSEQ_E_HIP;
    }
    int waves = opts && opts->waves > 0 ? opts->waves : kDefaultWaves;
    rc = ROTSEQ_E_UNSUPPORTED;
    while (waves >= 1 && (rc = set_waves(b, waves)) == ROTSEQ_E_UNSUPPORTED)
        --waves;
    if (rc == ROTSEQ_SUCCESS)
        rc = hipDeviceSynchronize() == hipSuccess ? ROTSEQ_SUCCESS : ROTSEQ_E_HIP;
    if (rc) {
        (void)hipFree(b->dmem);
        delete b;
        return rc;
    }
    *out = b;
    return ROTSEQ_SUCCESS;
}

int execute(rotseq_batch *b, hipStream_t stream)
{
    if (b == nullptr)
        return -1;
    if (b->L.count == 0)
        return ROTSEQ_SUCCESS;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev != b->device)
        return ROTSEQ_E_UNSUPPORTED;
    b->L.spin_limit = wait_spin_limit();
    b->L.wait_bias = wait_bias();
    if (launch_prep_batch(b->L, stream) != hipSuccess)
        return ROTSEQ_E_HIP;
    if (launch_chain_batch(b->L, stream) != hipSuccess)
        return ROTSEQ_E_HIP;
    return ROTSEQ_SUCCESS;
}

template <typename P>
int create_typed(int32_t count, const P *probs, const rotseq_opts *opts, rotseq_batch **out,
                 int esize)
{
    if (count < 0)
        return -1;
    if (count > 0 && probs == nullptr)
        return -2;
    std::vector<Entry> in;
    in.reserve(count);
    for (int32_t i = 0; i < count; ++i)
        in.push_back(entry_of(probs[i]));
    return create(count, in, esize, opts, out);
}

// New A, C and S pointers (and leading dimensions) for an existing plan:
// the same entries, in the order given at creation, with the same shapes.
int update(rotseq_batch *b, int32_t count, const std::vector<Entry> &in, int esize)
{
    if (b == nullptr)
        return -1;
    if (esize != b->esize || (size_t)count * 3 != b->shapes.size())
        return -2;
    for (int32_t i = 0; i < count; ++i) {
        const int64_t *sh = &b->shapes[(size_t)i * 3];
        if (in[i].m != sh[0])
            return -(1000 * (i + 1) + 1);
        if (in[i].n != sh[1])
            return -(1000 * (i + 1) + 2);
        if (in[i].k != sh[2])
            return -(1000 * (i + 1) + 3);
    }
    std::vector<int> work;
    const int bad = check_entries(count, in, esize, work);
    if (bad)
        return bad;
    std::vector<BatchItem> items = b->items;
    for (size_t t = 0; t < items.size(); ++t) {
        const Entry &e = in[b->order[t]];
        BatchItem &it = items[t];
        it.A = e.A;
        it.C = e.C;
        it.S = e.S;
        it.lda = e.lda;
        it.ldc = e.ldc;
        it.lds = e.lds;
    }
    if (items.empty())
        return ROTSEQ_SUCCESS;
    // The table is read by every execution, so none may be in flight.
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(b->dmem, items.data(), items.size() * sizeof(BatchItem), hipMemcpyHostToDevice) !=
            hipSuccess)
        return ROTSEQ_E_HIP;
    b->items.swap(items);
    return ROTSEQ_SUCCESS;
}

template <typename P>
int update_typed(rotseq_batch *b, int32_t count, const P *probs, int esize)
{
    if (b == nullptr)
        return -1;
    if (count < 0 || (count > 0 && probs == nullptr))
        return -2;
    std::vector<Entry> in;
    in.reserve(count);
    for (int32_t i = 0; i < count; ++i)
        in.push_back(entry_of(probs[i]));
    return update(b, count, in, esize);
}

// Reads the items' error words (device synchronized first) into `per_item`
// (dispatch order) and returns their OR; `reset` zeroes them afterwards.
int read_status(rotseq_batch *b, std::vector<int> &per_item, int reset)
{
    per_item.assign((size_t)b->L.count, 0);
    if (b->L.count == 0)
        return ROTSEQ_SUCCESS;
    char *words = (char *)b->dmem + b->L.status_off;
    const size_t bytes = (size_t)b->L.count * sizeof(int);
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(per_item.data(), words, bytes, hipMemcpyDeviceToHost) != hipSuccess)
        return -ROTSEQ_E_HIP;
    if (reset && (hipMemset(words, 0, bytes) != hipSuccess || hipDeviceSynchronize() != hipSuccess))
        return -ROTSEQ_E_HIP;
    int any = 0;
    for (int v : per_item)
        any |= v;
    return any;
}

template <typename P>
int one_shot(int32_t count, const P *probs, hipStream_t stream, int esize)
{
    rotseq_batch *b = nullptr;
    int rc = create_typed(count, probs, nullptr, &b, esize);
    if (rc)
        return rc;
    rc = execute(b, stream);
    if (hipStreamSynchronize(stream) != hipSuccess && rc == ROTSEQ_SUCCESS)
        rc = ROTSEQ_E_HIP;
    if (rc == ROTSEQ_SUCCESS) {
        // A bounded wait that gave up leaves wrong results: report it.
        std::vector<int> words;
        const int any = read_status(b, words, 0);
        if (any < 0)
            rc = -any;
        else if (any != 0)
            rc = ROTSEQ_E_TIMEOUT;
    }
    (void)hipFree(b->dmem);
    delete b;
    return rc;
}

}  // namespace
}  // namespace rotseq

using namespace rotseq;

extern "C" {

int rotseq_batch_create_d(int32_t count, const rotseq_problem_d *probs, const rotseq_opts *opts,
                          rotseq_batch **out)
{
    return create_typed(count, probs, opts, out, 8);
}

int rotseq_batch_create_s(int32_t count, const rotseq_problem_s *probs, const rotseq_opts *opts,
                          rotseq_batch **out)
{
    return create_typed(count, probs, opts, out, 4);
}

int rotseq_batch_execute(rotseq_batch *batch, hipStream_t stream) { return execute(batch, stream); }

int rotseq_batch_update_d(rotseq_batch *batch, int32_t count, const rotseq_problem_d *probs)
{
    return update_typed(batch, count, probs, 8);
}

int rotseq_batch_update_s(rotseq_batch *batch, int32_t count, const rotseq_problem_s *probs)
{
    return update_typed(batch, count, probs, 4);
}

int rotseq_batch_tune(rotseq_batch *b, hipStream_t stream, int32_t reps)
{
    if (b == nullptr)
        return -1;
    if (reps < 1)
        return -3;
    if (b->L.count == 0)
        return ROTSEQ_SUCCESS;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return ROTSEQ_E_HIP;
    int best_waves = b->L.waves;
    float best = 1e30f;
    int rc = ROTSEQ_SUCCESS;
    for (int w : kTuneWaves) {
        if (set_waves(b, w) != ROTSEQ_SUCCESS)
            continue;
        if ((rc = execute(b, stream)) != ROTSEQ_SUCCESS)
            break;
        (void)hipEventRecord(e0, stream);
        for (int r = 0; r < reps && rc == ROTSEQ_SUCCESS; ++r)
            rc = execute(b, stream);
        (void)hipEventRecord(e1, stream);
        float ms = 0.f;
        if (rc || hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            rc = rc ? rc : ROTSEQ_E_HIP;
            break;
        }
        if (ms < best) {
            best = ms;
            best_waves = w;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    const int rc2 = set_waves(b, best_waves);
    return rc ? rc : rc2;
}

int rotseq_batch_status(rotseq_batch *b, int32_t *per_problem, int reset)
{
    if (b == nullptr)
        return -1;
    std::vector<int> words;
    const int any = read_status(b, words, reset);
    if (any < 0)
        return -any;
    if (per_problem) {
        for (size_t i = 0; i < b->shapes.size() / 3; ++i)
            per_problem[i] = 0;
        for (size_t t = 0; t < words.size(); ++t)
            per_problem[b->order[t]] = words[t] & 0xff;  // ROTSEQ_E_* code
    }
    return any ? ROTSEQ_E_TIMEOUT : ROTSEQ_SUCCESS;
}

int rotseq_batch_info_get(const rotseq_batch *b, rotseq_batch_info *info)
{
    if (b == nullptr)
        return -1;
    if (info == nullptr)
        return -2;
    *info = rotseq_batch_info{};
    info->count = b->L.count;
    info->band = b->L.band;
    info->waves = b->L.waves;
    info->workgroups = b->L.nwg;
    info->waves_total = b->waves_total;
    info->flops = b->flops;
    info->bytes = b->bytes;
    info->device_bytes = b->dbytes;
    return ROTSEQ_SUCCESS;
}

int rotseq_batch_destroy(rotseq_batch *b)
{
    if (b == nullptr)
        return ROTSEQ_SUCCESS;
    int rc = hipDeviceSynchronize() == hipSuccess ? ROTSEQ_SUCCESS : ROTSEQ_E_HIP;
    if (hipFree(b->dmem) != hipSuccess)
        rc = ROTSEQ_E_HIP;
    delete b;
    return rc;
}

int rotseq_batched_d(int32_t count, const rotseq_problem_d *probs, hipStream_t stream)
{
    return one_shot(count, probs, stream, 8);
}

int rotseq_batched_s(int32_t count, const rotseq_problem_s *probs, hipStream_t stream)
{
    return one_shot(count, probs, stream, 4);
}

}  // extern "C"
