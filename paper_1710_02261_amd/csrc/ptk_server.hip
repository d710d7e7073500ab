// Serving loop: continuous batching of fold-in solves and predictions on a
// bound model (the row update of eq. "rowupdate" for rows that are not in
// the model, and eq. "recon2" for missing entries).
//
// A library thread owns S slots; each slot has its own stream, a device
// arena, pinned staging memory and an event. Requests are copied at submit
// and admitted first-in first-out while they fit in a slot's memory. While
// one slot's batch runs on the GPU, the next idle slot packs the requests
// that arrived meanwhile and launches them on its own stream, so batches
// overlap on the device and each slot's memory is reused as soon as its
// batch completes.
//
// A batch of fold-ins of mode n is laid out as the rows of a small CSR: one
// row per request, its entries padded to a multiple of 64 so that every
// request starts a work range of 64 entries. The row systems are formed by
// the same delta/Gram kernel as the ALS sweep (padding entries belong to a
// row whose sums are discarded), rows longer than one range are merged in
// range order, and the FP64 solve writes the new rows. The arithmetic
// applied to a request therefore depends only on its own entries: a result
// is bitwise the same alone and in any mix. Predictions of a batch run as one
// per-entry launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "ptk_context.h"
#include "ptk_internal.h"

using namespace ptk;

namespace {

constexpr int64_t kSeg = 64;            // fold-in segment / work-range size
constexpr size_t kAlign = 256;
constexpr size_t kBatchSlack = 1 << 20; // per-batch layout overhead bound
using Clock = std::chrono::steady_clock;

struct Request {
    uint64_t ticket = 0;
    int kind = 0;                       // 0 fold-in, 1 predict
    int32_t mode = 0;
    int64_t count = 0;                  // k or m
    std::vector<int32_t> idx;           // [N][count]
    std::vector<float> val;             // [count] (fold-in)
    size_t bytes = 0;
    ptk_status status = PTK_OK;
    std::vector<float> out;
    bool done = false;
    Clock::time_point t_submit, t_done;
};
using ReqPtr = std::shared_ptr<Request>;

struct Slot {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    char *dev = nullptr;
    char *host = nullptr;
    int32_t *bad = nullptr;     // least-squares solve counters [3]
    bool busy = false;
    std::vector<ReqPtr> reqs;
    std::vector<size_t> out_off;
    size_t out_begin = 0, out_end = 0;
};

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

__global__ void k_fill_nan(float *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = __builtin_nanf("");
}

}  // namespace

struct ptk_server {
    ptk_ctx *ctx = nullptr;
    ptk_server_opts opt{};
    Shape s{};
    int device = 0;
    double *gp[kMaxN] = {};             // fp64 permuted core per mode
    bool fast[kMaxN] = {};
    std::vector<Slot> slots;
    size_t slot_cap = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<ReqPtr> queue;
    std::unordered_map<uint64_t, ReqPtr> table;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread worker;
    ptk_server_stats stats{};
    std::string err;
};

namespace {

ptk_status sfail(ptk_server *sv, ptk_status s, const std::string &msg) {
    if (sv) sv->err = msg;
    return s;
}

// Least-squares lists of a group of q fold-in rows over P entries: counters
// [4], the row list [q], heavy rows and first tasks [2q], a flag byte per
// row. Tasks of
// kServeTaskLen entries: at most P / 64 + 1 of them, whose triangles fit in
// the group's partial systems ((P / kSeg + 1) * 2 * E doubles, free after
// the merge).
constexpr int32_t kServeTaskLen = 128;
int64_t ls_tcap(int64_t P) { return 2 * (P / kServeTaskLen) + 1; }
int64_t ls_ints(int64_t q, int64_t) { return 4 + 3 * q + (q + 3) / 4; }

size_t request_bytes(const ptk_server *sv, const Request &r) {
    const int N = sv->s.N;
    if (r.kind == 1) return align_up((size_t)r.count * (4 * N + 4)) + 2 * kAlign;
    const int J = sv->s.ranks[r.mode];
    const size_t E = sys_entries(J);
    const size_t P = (size_t)((r.count + kSeg - 1) / kSeg * kSeg);
    const size_t chunks = P / kSeg;
    return P * (4 * (N - 1) + 8) + J * 4 + E * 8 + chunks * 2 * E * 8 + chunks * 12 +
           16 + ls_ints(1, (int64_t)P) * 4 + 9 * kAlign;
}

// Bump allocator over a slot's arena (same offsets in staging and device).
struct Layout {
    size_t off = 0;
    size_t take(size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes);
        return o;
    }
};

// Pack the slot's requests, copy them in, launch, copy results out, record.
hipError_t launch_batch(ptk_server *sv, Slot &sl) {
    const Shape &s = sv->s;
    const int N = s.N;
    ptk_ctx *c = sv->ctx;
    Layout L;
    // inputs first (one host-to-device copy), then device-only buffers, then
    // outputs (one device-to-host copy)
    struct Group {
        int n = 0;
        std::vector<size_t> ri;         // indices into sl.reqs
        int64_t P = 0;
        size_t o_oidx = 0, o_val = 0, o_rows = 0, o_rowptr = 0, o_split = 0;
        size_t o_ls = 0;                // least-squares lists (ls_ints)
        size_t o_bbuf = 0, o_part = 0, o_out = 0;
        int32_t nsplit = 0;
    };
    std::vector<Group> groups;
    std::vector<size_t> pred;
    for (size_t i = 0; i < sl.reqs.size(); ++i) {
        const Request &r = *sl.reqs[i];
        if (r.kind == 1) {
            pred.push_back(i);
            continue;
        }
        auto it = std::find_if(groups.begin(), groups.end(),
                               [&](const Group &g) { return g.n == r.mode; });
        if (it == groups.end()) {
            groups.push_back(Group());
            groups.back().n = r.mode;
            it = groups.end() - 1;
        }
        it->ri.push_back(i);
    }
    int64_t M = 0;
    for (size_t i : pred) M += sl.reqs[i]->count;
    for (Group &g : groups) {
        for (size_t i : g.ri) g.P += (sl.reqs[i]->count + kSeg - 1) / kSeg * kSeg;
        const int64_t q = (int64_t)g.ri.size();
        g.o_oidx = L.take((size_t)(N - 1) * g.P * 4);
        g.o_val = L.take((size_t)g.P * 4);
        g.o_rows = L.take((size_t)g.P * 4);
        g.o_rowptr = L.take((size_t)(q + 2) * 8);
        g.o_split = L.take((size_t)(g.P / kSeg + 1) * 12);
        g.o_ls = L.take((size_t)ls_ints(q, g.P) * 4);
    }
    const size_t o_pidx = L.take((size_t)N * M * 4);
    const size_t in_end = L.off;
    for (Group &g : groups) {
        const int64_t q = (int64_t)g.ri.size();
        const size_t E = sys_entries(s.ranks[g.n]);
        g.o_bbuf = L.take((size_t)(q + 1) * E * 8);
        g.o_part = L.take((size_t)(g.P / kSeg + 1) * 2 * E * 8);
    }
    sl.out_begin = L.off;
    for (Group &g : groups) g.o_out = L.take((size_t)g.ri.size() * s.ranks[g.n] * 4);
    const size_t o_pout = L.take((size_t)M * 4);
    sl.out_end = L.off;
    if (sl.out_end > sv->slot_cap) return hipErrorOutOfMemory;   // admission bug guard

    // fill the staging copy of the inputs
    char *H = sl.host;
    for (Group &g : groups) {
        int32_t *oidx = (int32_t *)(H + g.o_oidx);
        float *val = (float *)(H + g.o_val);
        int32_t *rows = (int32_t *)(H + g.o_rows);
        int64_t *rowptr = (int64_t *)(H + g.o_rowptr);
        int32_t *split = (int32_t *)(H + g.o_split);
        const int64_t q = (int64_t)g.ri.size();
        int64_t pos = 0;
        g.nsplit = 0;
        for (int64_t i = 0; i < q; ++i) {
            const Request &r = *sl.reqs[g.ri[i]];
            const int64_t k = r.count, P = (k + kSeg - 1) / kSeg * kSeg;
            rowptr[i] = pos;
            int t = 0;
            for (int m = 0; m < N; ++m) {
                if (m == g.n) continue;
                int32_t *dst = oidx + (int64_t)t * g.P + pos;
                std::memcpy(dst, r.idx.data() + (size_t)m * k, (size_t)k * 4);
                std::memset(dst + k, 0, (size_t)(P - k) * 4);
                ++t;
            }
            std::memcpy(val + pos, r.val.data(), (size_t)k * 4);
            std::memset(val + pos + k, 0, (size_t)(P - k) * 4);
            for (int64_t e = 0; e < k; ++e) rows[pos + e] = (int32_t)i;
            for (int64_t e = k; e < P; ++e) rows[pos + e] = (int32_t)q;   // padding row
            if (P > kSeg) {
                split[3 * g.nsplit + 0] = (int32_t)i;
                split[3 * g.nsplit + 1] = (int32_t)(pos / kSeg);
                split[3 * g.nsplit + 2] = (int32_t)((pos + k - 1) / kSeg);
                ++g.nsplit;
            }
            pos += P;
        }
        rowptr[q] = pos;
        rowptr[q + 1] = pos;
        int32_t *ls = (int32_t *)(H + g.o_ls);
        for (int k = 0; k < 4; ++k) ls[k] = 0;      // no row flagged yet
    }
    {
        int32_t *pidx = (int32_t *)(H + o_pidx);
        int64_t off = 0;
        for (size_t i : pred) {
            const Request &r = *sl.reqs[i];
            for (int m = 0; m < N; ++m)
                std::memcpy(pidx + (int64_t)m * M + off, r.idx.data() + (size_t)m * r.count,
                            (size_t)r.count * 4);
            off += r.count;
        }
    }
    hipError_t e = hipSuccess;
    if (in_end) e = hipMemcpyAsync(sl.dev, sl.host, in_end, hipMemcpyHostToDevice, sl.st);
    char *D = sl.dev;
    for (Group &g : groups) {
        if (e != hipSuccess) break;
        const int n = g.n;
        const int J = s.ranks[n];
        const int64_t q = (int64_t)g.ri.size();
        float *out = (float *)(D + g.o_out);
        hipLaunchKernelGGL(k_fill_nan, dim3((unsigned)((q * J + 255) / 256)), dim3(256), 0,
                           sl.st, out, q * J);
        if ((e = hipGetLastError()) != hipSuccess) break;
        GramArgs a{};
        int t = 0, offj = 0;
        for (int m = 0; m < N; ++m) {
            if (m == n) continue;
            a.fac[t] = c->fac[m];
            a.oidx[t] = (const int32_t *)(D + g.o_oidx) + (int64_t)t * g.P;
            a.jk[t] = s.ranks[m];
            a.aoff[t] = offj;
            offj += s.ranks[m];
            ++t;
        }
        a.gp = sv->gp[n];
        a.nother = N - 1;
        a.jn = J;
        a.E = sys_entries(J);
        a.rows = (const int32_t *)(D + g.o_rows);
        a.skip_row = (int32_t)q;
        a.val = (const float *)(D + g.o_val);
        a.rowptr = (const int64_t *)(D + g.o_rowptr);
        a.nnz = g.P;
        a.chunk = kSeg;
        a.bbuf = (double *)(D + g.o_bbuf);
        a.part = (double *)(D + g.o_part);
        e = launch_gram(a, s, n, kArithF64, g.P / kSeg, sv->fast[n], sl.st);
        if (e == hipSuccess)
            e = launch_merge(a.part, (const int32_t *)(D + g.o_split), g.nsplit, a.E, a.bbuf,
                             sl.st);
        // rows whose Cholesky solve would be inaccurate go to the
        // least-squares form; the triangles of their tasks reuse part
        SolveFlags f{};
        int32_t *ls = (int32_t *)(D + g.o_ls);
        f.rflag = (uint8_t *)(ls + 4 + 3 * q);
        f.cnt = ls;
        f.list = ls + 4;
        f.cap = q;
        f.hrow = ls + 4 + q;
        f.hoff = ls + 4 + 2 * q;
        f.hcap = q;
        f.tcap = ls_tcap(g.P);
        f.task_len = kServeTaskLen;
        f.pack = J < kLsPack;
        f.cond_limit = c->opt.cond_limit > 0.0 ? c->opt.cond_limit : kCondLimitDefault;
        if (e == hipSuccess)
            e = launch_solve(a.bbuf, a.rowptr, q, J, sv->opt.lambda, out, f, sl.st);
        if (e == hipSuccess) e = launch_ls_lists(a.rowptr, q, f, sl.st);
        if (e == hipSuccess) {
            LsArgs r{};
            r.gp = a.gp;
            for (int k = 0; k < N - 1; ++k) {
                r.fac[k] = a.fac[k];
                r.oidx[k] = a.oidx[k];
                r.jk[k] = a.jk[k];
                r.aoff[k] = a.aoff[k];
            }
            r.nother = N - 1;
            r.jn = J;
            r.val = a.val;
            r.rowptr = a.rowptr;
            r.f = f;
            r.tri = a.part;
            r.lambda = sv->opt.lambda;
            r.A = out;
            r.rsse = nullptr;
            r.stats = sl.bad;
            e = launch_ls(r, N, sv->fast[n], c->num_cu, sl.st);
        }
    }
    if (e == hipSuccess && M > 0) {
        EntryArgs a{};
        const int32_t *pidx = (const int32_t *)(D + o_pidx);
        int offj = 0;
        for (int m = 1; m < N; ++m) {
            a.fac[m - 1] = c->fac[m];
            a.oidx[m - 1] = pidx + (int64_t)m * M;
            a.jk[m - 1] = s.ranks[m];
            a.aoff[m - 1] = offj;
            offj += s.ranks[m];
        }
        a.gp = sv->gp[0];
        a.nother = N - 1;
        a.jn = s.ranks[0];
        a.own_idx = pidx;
        a.own = c->fac[0];
        a.m = M;
        a.out = (float *)(D + o_pout);
        const int64_t blocks = std::min<int64_t>((M + kWave - 1) / kWave, 4096);
        e = launch_entries(a, s, 0, kOutPredict, sv->fast[0], blocks, sl.st);
    }
    // request outputs in staging
    sl.out_off.assign(sl.reqs.size(), 0);
    for (Group &g : groups)
        for (size_t i = 0; i < g.ri.size(); ++i)
            sl.out_off[g.ri[i]] = g.o_out + i * (size_t)s.ranks[g.n] * 4;
    {
        size_t off = o_pout;
        for (size_t i : pred) {
            sl.out_off[i] = off;
            off += (size_t)sl.reqs[i]->count * 4;
        }
    }
    if (e == hipSuccess && sl.out_end > sl.out_begin)
        e = hipMemcpyAsync(sl.host + sl.out_begin, sl.dev + sl.out_begin,
                           sl.out_end - sl.out_begin, hipMemcpyDeviceToHost, sl.st);
    if (e == hipSuccess) e = hipEventRecord(sl.ev, sl.st);
    return e;
}

void complete_batch(ptk_server *sv, Slot &sl, hipError_t e) {
    const Clock::time_point now = Clock::now();
    std::lock_guard<std::mutex> lk(sv->mu);
    for (size_t i = 0; i < sl.reqs.size(); ++i) {
        Request &r = *sl.reqs[i];
        if (e != hipSuccess) {
            r.status = PTK_E_HIP;
        } else {
            const size_t n = r.kind == 1 ? (size_t)r.count : (size_t)sv->s.ranks[r.mode];
            r.out.resize(n);
            std::memcpy(r.out.data(), sl.host + sl.out_off[i], n * 4);
            if (r.kind == 0)
                for (float v : r.out)
                    if (std::isnan(v)) r.status = PTK_E_NOT_PD;
        }
        r.done = true;
        r.t_done = now;
        r.idx.clear();
        r.idx.shrink_to_fit();
        r.val.clear();
        r.val.shrink_to_fit();
        sv->stats.requests += 1;
    }
    sv->stats.batches += 1;
    sv->stats.max_batch_requests =
        std::max<int64_t>(sv->stats.max_batch_requests, (int64_t)sl.reqs.size());
    sl.reqs.clear();
    sl.busy = false;
    sv->cv_done.notify_all();
}

void worker_main(ptk_server *sv) {
    (void)hipSetDevice(sv->device);
    for (;;) {
        bool progressed = false;
        for (Slot &sl : sv->slots) {
            if (!sl.busy) continue;
            const hipError_t q = hipEventQuery(sl.ev);
            if (q == hipErrorNotReady) continue;
            complete_batch(sv, sl, q);
            progressed = true;
        }
        Slot *idle = nullptr;
        for (Slot &sl : sv->slots)
            if (!sl.busy) {
                idle = &sl;
                break;
            }
        bool any_busy = false;
        for (Slot &sl : sv->slots) any_busy |= sl.busy;
        if (idle) {
            std::unique_lock<std::mutex> lk(sv->mu);
            size_t used = kBatchSlack;
            while (!sv->queue.empty() &&
                   (int64_t)idle->reqs.size() < sv->opt.max_batch_requests) {
                const ReqPtr &r = sv->queue.front();
                if (used + r->bytes > sv->slot_cap) break;   // FIFO admission by memory
                used += r->bytes;
                idle->reqs.push_back(r);
                sv->queue.pop_front();
            }
            if (!idle->reqs.empty()) {
                idle->busy = true;
                int64_t inflight = 0;
                for (Slot &q : sv->slots) inflight += q.busy ? 1 : 0;
                sv->stats.max_in_flight = std::max(sv->stats.max_in_flight, inflight);
                lk.unlock();
                const hipError_t e = launch_batch(sv, *idle);
                if (e != hipSuccess) {
                    (void)hipStreamSynchronize(idle->st);
                    complete_batch(sv, *idle, e);
                }
                progressed = true;
                any_busy = true;
            } else if (!any_busy) {
                if (sv->stop && sv->queue.empty()) break;
                sv->cv_work.wait_for(lk, std::chrono::milliseconds(2));
                continue;
            }
        }
        if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
}

ptk_status validate_and_copy(ptk_server *sv, Request &r, const int32_t *idx,
                             const float *val) {
    const int N = sv->s.N;
    r.idx.resize((size_t)N * r.count);
    for (int m = 0; m < N; ++m) {
        const int32_t *src = idx + (size_t)m * r.count;
        int32_t *dst = r.idx.data() + (size_t)m * r.count;
        if (r.kind == 0 && m == r.mode) {        // not read for a fold-in
            std::memset(dst, 0, (size_t)r.count * 4);
            continue;
        }
        const int64_t I = sv->s.dims[m];
        for (int64_t e = 0; e < r.count; ++e) {
            if (src[e] < 0 || src[e] >= I)
                return sfail(sv, PTK_E_INVALID, "index out of range in request");
            dst[e] = src[e];
        }
    }
    if (r.kind == 0) {
        r.val.assign(val, val + r.count);
        for (float v : r.val)
            if (!std::isfinite(v)) return sfail(sv, PTK_E_INVALID, "non-finite value in request");
    }
    return PTK_OK;
}

ptk_status submit(ptk_server *sv, ReqPtr r, uint64_t *ticket) {
    r->bytes = request_bytes(sv, *r);
    if (r->bytes + kBatchSlack > sv->slot_cap)
        return sfail(sv, PTK_E_NOMEM, "request larger than a slot's memory budget");
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stop) return sfail(sv, PTK_E_STATE, "server is shutting down");
    if ((int64_t)sv->queue.size() >= sv->opt.queue_capacity)
        return sfail(sv, PTK_E_BUSY, "request queue is full");
    r->ticket = sv->next_ticket++;
    r->t_submit = Clock::now();
    sv->queue.push_back(r);
    sv->table[r->ticket] = r;
    *ticket = r->ticket;
    sv->cv_work.notify_one();
    return PTK_OK;
}

ptk_status take_result(ptk_server *sv, Request &r, float *out, int64_t cap,
                       ptk_status *req_status, double *latency_ms) {
    if (out) {
        const int64_t n = std::min<int64_t>(cap, (int64_t)r.out.size());
        if (n > 0) std::memcpy(out, r.out.data(), (size_t)n * 4);
    }
    if (req_status) *req_status = r.status;
    if (latency_ms)
        *latency_ms =
            std::chrono::duration<double, std::milli>(r.t_done - r.t_submit).count();
    sv->table.erase(r.ticket);
    return PTK_OK;
}

}  // namespace

extern "C" {

ptk_status ptk_server_create(ptk_server **out, ptk_ctx *ctx, const ptk_server_opts *o) {
    if (!out || !ctx || !o) return PTK_E_INVALID;
    *out = nullptr;
    if (!ctx->core) return PTK_E_STATE;
    if (!(o->lambda > 0.0) || o->slots < 0 || o->mem_budget_bytes < 0 ||
        o->max_batch_requests < 0 || o->queue_capacity < 0)
        return PTK_E_INVALID;
    std::unique_ptr<ptk_server> sv(new (std::nothrow) ptk_server());
    if (!sv) return PTK_E_NOMEM;
    sv->ctx = ctx;
    sv->opt = *o;
    if (sv->opt.slots == 0) sv->opt.slots = 2;
    if (sv->opt.mem_budget_bytes == 0) sv->opt.mem_budget_bytes = (int64_t)512 << 20;
    if (sv->opt.max_batch_requests == 0) sv->opt.max_batch_requests = 4096;
    if (sv->opt.queue_capacity == 0) sv->opt.queue_capacity = 1 << 20;
    sv->s = ctx->s;
    sv->device = ctx->device;
    sv->slot_cap = align_up((size_t)(sv->opt.mem_budget_bytes / sv->opt.slots));
    if (sv->slot_cap < 2 * kBatchSlack) return PTK_E_INVALID;
    const int N = sv->s.N;
    bool eq = true;
    for (int k = 1; k < N; ++k) eq &= sv->s.ranks[k] == sv->s.ranks[0];
    hipError_t e = hipSuccess;
    for (int n = 0; n < N && e == hipSuccess; ++n) {
        sv->fast[n] = eq && fast_available(N, sv->s.ranks[n], kArithF64);
        e = hipMalloc((void **)&sv->gp[n], (size_t)(ctx->core_cells + 64) * 8);
        if (e == hipSuccess)
            e = launch_permute_core(ctx->core, sv->gp[n], sv->s, n, kArithF64, ctx->st);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->st);
    sv->slots.resize(sv->opt.slots);
    for (Slot &sl : sv->slots) {
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming);
        if (e == hipSuccess) e = hipMalloc((void **)&sl.dev, sv->slot_cap);
        if (e == hipSuccess) e = hipHostMalloc((void **)&sl.host, sv->slot_cap);
        if (e == hipSuccess) e = hipMalloc((void **)&sl.bad, 4 * sizeof(int32_t));
        if (e == hipSuccess) e = hipMemset(sl.bad, 0, 4 * sizeof(int32_t));
    }
    if (e != hipSuccess) {
        ptk_server_destroy(sv.release());
        return e == hipErrorOutOfMemory ? PTK_E_NOMEM : PTK_E_HIP;
    }
    ptk_server *p = sv.release();
    p->worker = std::thread(worker_main, p);
    *out = p;
    return PTK_OK;
}

ptk_status ptk_server_submit_foldin(ptk_server *sv, int32_t n, int64_t k,
                                    const int32_t *idx_host, const float *val_host,
                                    uint64_t *ticket) {
    if (!sv || !ticket) return PTK_E_INVALID;
    if (n < 0 || n >= sv->s.N) return sfail(sv, PTK_E_INVALID, "mode out of range");
    if (k < 0 || k >= (int64_t(1) << 31)) return sfail(sv, PTK_E_INVALID, "k out of range");
    if (k > 0 && (!idx_host || !val_host)) return sfail(sv, PTK_E_INVALID, "null input");
    auto r = std::make_shared<Request>();
    r->kind = 0;
    r->mode = n;
    r->count = k;
    ptk_status st = validate_and_copy(sv, *r, idx_host, val_host);
    if (st != PTK_OK) return st;
    return submit(sv, r, ticket);
}

ptk_status ptk_server_submit_predict(ptk_server *sv, int64_t m, const int32_t *idx_host,
                                     uint64_t *ticket) {
    if (!sv || !ticket) return PTK_E_INVALID;
    if (m < 0 || m >= (int64_t(1) << 31)) return sfail(sv, PTK_E_INVALID, "m out of range");
    if (m > 0 && !idx_host) return sfail(sv, PTK_E_INVALID, "null input");
    auto r = std::make_shared<Request>();
    r->kind = 1;
    r->count = m;
    ptk_status st = validate_and_copy(sv, *r, idx_host, nullptr);
    if (st != PTK_OK) return st;
    return submit(sv, r, ticket);
}

ptk_status ptk_server_poll(ptk_server *sv, uint64_t ticket, float *out_host, int64_t cap,
                           int32_t *done, ptk_status *req_status, double *latency_ms) {
    if (!sv || !done) return PTK_E_INVALID;
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->table.find(ticket);
    if (it == sv->table.end()) return sfail(sv, PTK_E_INVALID, "unknown ticket");
    ReqPtr r = it->second;
    *done = r->done ? 1 : 0;
    if (!r->done) return PTK_OK;
    return take_result(sv, *r, out_host, cap, req_status, latency_ms);
}

ptk_status ptk_server_wait(ptk_server *sv, uint64_t ticket, float *out_host, int64_t cap,
                           double timeout_s, ptk_status *req_status, double *latency_ms) {
    if (!sv) return PTK_E_INVALID;
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->table.find(ticket);
    if (it == sv->table.end()) return sfail(sv, PTK_E_INVALID, "unknown ticket");
    ReqPtr r = it->second;
    const auto deadline = Clock::now() + std::chrono::duration_cast<Clock::duration>(
                                             std::chrono::duration<double>(timeout_s));
    while (!r->done) {
        if (sv->cv_done.wait_until(lk, deadline) == std::cv_status::timeout && !r->done)
            return sfail(sv, PTK_E_BUSY, "timed out waiting for the request");
    }
    return take_result(sv, *r, out_host, cap, req_status, latency_ms);
}

ptk_status ptk_server_get_stats(ptk_server *sv, ptk_server_stats *out) {
    if (!sv || !out) return PTK_E_INVALID;
    std::lock_guard<std::mutex> lk(sv->mu);
    *out = sv->stats;
    out->queued = (int64_t)sv->queue.size();
    return PTK_OK;
}

const char *ptk_server_last_error(const ptk_server *sv) {
    if (!sv) return "null server";
    return sv->err.c_str();
}

ptk_status ptk_server_destroy(ptk_server *sv) {
    if (!sv) return PTK_OK;
    if (sv->worker.joinable()) {
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            sv->stop = true;
        }
        sv->cv_work.notify_all();
        sv->worker.join();
    }
    for (Slot &sl : sv->slots) {
        if (sl.st) (void)hipStreamSynchronize(sl.st);
        if (sl.dev) (void)hipFree(sl.dev);
        if (sl.host) (void)hipHostFree(sl.host);
        if (sl.bad) (void)hipFree(sl.bad);
        if (sl.ev) (void)hipEventDestroy(sl.ev);
        if (sl.st) (void)hipStreamDestroy(sl.st);
    }
    for (int n = 0; n < kMaxN; ++n)
        if (sv->gp[n]) (void)hipFree(sv->gp[n]);
    delete sv;
    return PTK_OK;
}

}  // extern "C"
