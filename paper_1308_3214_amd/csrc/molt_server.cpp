// Request server: many independent solves of differing size and order served
// concurrently on one GPU.  Requests are admitted in arrival order while their
// device footprint (plan workspace, line-object tables, two state fields) fits
// a byte budget; an admitted request keeps its fields resident in HBM, runs
// start + (nsteps - 1) steps from its own captured hipGraph on one stream of a
// pool (default priority; requests on different streams overlap on the
// hardware queues), and signals completion with an event.  All allocations of
// a request are stream-ordered, so admitting and retiring requests never
// synchronises the device.
//
// Batched mode: admitted requests advance in rounds of one step each on one
// stream.  A round gathers the launches of every running request's step,
// groups them by position in the step and kernel instantiation, writes the
// argument sets of each group into one table (pinned staging, one copy per
// round) and runs each group as one batched launch; masked requests' launches
// run one by one in their position.  Three staging slots bound the rounds in
// flight.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/molt.h"
#include "molt_program.h"

namespace {

enum ReqState { Q_QUEUED = 0, Q_RUNNING = 1, Q_DONE = 2, Q_FAILED = 3 };

struct Req {
    int64_t id = 0;
    mol_desc desc{};
    std::vector<uint8_t> mask;
    std::vector<double> cross;
    const void *u0 = nullptr;
    bool u0_dev = false;
    int64_t nsteps = 0;
    size_t footprint = 0;     // bytes held while running
    size_t field = 0;         // bytes of one field (held until the result is taken)
    ReqState state = Q_QUEUED;
    bool reported = false;    // returned by a poll
    mol_plan *plan = nullptr;
    void *d_prev = nullptr, *d_curr = nullptr;
    int stream = 0;
    double work = 0;          // point-updates of the request (stream load estimate)
    int64_t left = 0;         // batched mode: steps still to run
    int par = 0;              // batched mode: buffer roles of the next step
    bool recorded = false;    // batched mode: completion event recorded
    // batched mode: argument sets of the step's launches for both buffer roles
    struct Cached {
        int k;
        molt::SweepKey key;
        int64_t blocks;
        size_t off, bytes;
    };
    std::vector<Cached> ops[2];
    std::vector<unsigned char> args[2];
    // launches that cannot share a batched table (line objects of a mask,
    // L^{-1} sweeps, the two-pass exact sweeps) run one by one in their position
    bool direct = false;
    hipEvent_t done = nullptr;
    std::string err;
};

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct mol_server_ {
    size_t budget = 0, used = 0, peak = 0;
    std::vector<hipStream_t> streams;
    std::vector<double> load;         // outstanding point-updates per stream
    hipStream_t copy = nullptr;       // results leave, and finished requests' memory
                                      // returns to the pool, on their own stream
    // device memory of the requests and round tables; what is freed stays
    // reserved in the pool (no release threshold), so that admitting a
    // request costs no allocation from the driver once the pool has grown
    hipMemPool_t pool = nullptr;
    int64_t next_id = 1;
    std::deque<Req *> queue;
    std::map<int64_t, Req *> reqs;
    int64_t completed = 0;
    std::mutex mu;
    double t0 = 0;
    double admit_s = 0;               // host time spent admitting requests
    double admit_max_s = 0;
    // batched mode
    bool batched = false;
    struct Slot {
        void *h = nullptr;                // pinned staging
        void *d = nullptr;                // device table
        size_t cap = 0;
        hipEvent_t ev = nullptr;          // after the slot's copy
        bool used = false;
    };
    static constexpr int NSLOT = 3;
    Slot slots[NSLOT];
    int64_t rounds = 0, launches = 0, sweeps = 0;
    double round_s = 0;               // host time spent issuing rounds
};

namespace {

thread_local std::string s_err;

mol_status sfail(mol_status s, const std::string &m)
{
    s_err = m;
    return s;
}

size_t elem_size(const mol_desc &d) { return d.dtype == MOL_F64 ? 8 : 4; }

int64_t npoints(const mol_desc &d)
{
    int64_t n = 1;
    for (int a = 0; a < d.ndim; ++a) n *= d.n[a];
    return n;
}

// Release everything but the result field.  The request's work is complete
// (its event fired, or its stream was synchronised), so the memory goes back
// to the pool on the copy stream, which holds no pending work here: freed at
// the tail of the request's own stream it would be ordered after the solves
// queued there since, and a request on another stream that is handed the
// same memory by the pool would wait for all of them.
void retire(mol_server_ *s, Req *r)
{
    hipStream_t st = s->copy;
    s->load[r->stream] -= r->work;
    r->work = 0;
    if (r->plan) molt::plan_destroy_async(r->plan, st);
    r->plan = nullptr;
    if (r->d_prev) (void)hipFreeAsync(r->d_prev, st);
    r->d_prev = nullptr;
    if (r->done) (void)hipEventDestroy(r->done);
    r->done = nullptr;
    s->used -= (r->footprint - r->field);
}

// Launch an admitted request on its stream.
mol_status launch(mol_server_ *s, Req *r)
{
    // the stream with the least outstanding work: a short request does not
    // queue behind a long one when another stream is free
    int best = 0;
    for (int i = 1; i < (int)s->streams.size(); ++i)
        if (s->load[i] < s->load[best]) best = i;
    r->stream = best;
    r->work = (double)npoints(r->desc) * (double)r->nsteps * (double)r->desc.P;
    s->load[best] += r->work;
    hipStream_t st = s->streams[r->stream];
    mol_desc d = r->desc;
    d.mask = r->mask.empty() ? nullptr : r->mask.data();
    d.cross = r->cross.empty() ? nullptr : r->cross.data();
    mol_status ms = molt::plan_create_async(&d, st, &r->plan, s->pool);
    if (ms != MOL_OK) return sfail(ms, mol_last_error());
    if (hipMallocFromPoolAsync(&r->d_prev, r->field, s->pool, st) != hipSuccess ||
        hipMallocFromPoolAsync(&r->d_curr, r->field, s->pool, st) != hipSuccess)
        return sfail(MOL_E_NOMEM, "stream-ordered allocation of the state fields failed");
    if (hipMemcpyAsync(r->d_prev, r->u0, r->field,
                       r->u0_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                       st) != hipSuccess)
        return sfail(MOL_E_DEVICE, "copy of the initial field failed");
    ms = mol_start(r->plan, r->d_prev, nullptr, r->d_curr, st);
    if (ms == MOL_OK && r->nsteps > 1) ms = mol_solve(r->plan, r->d_prev, r->d_curr, r->nsteps - 1, st);
    if (ms != MOL_OK) return sfail(ms, mol_last_error());
    if (hipEventCreateWithFlags(&r->done, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(r->done, st) != hipSuccess)
        return sfail(MOL_E_DEVICE, "completion event failed");
    return MOL_OK;
}

// Batched mode: allocations, initial field, start step and (fused solves) the
// first D_x of the solve on the round stream; the request then joins the
// rounds.
mol_status admit_batched(mol_server_ *s, Req *r)
{
    r->stream = 0;
    hipStream_t st = s->streams[0];
    mol_desc d = r->desc;
    d.mask = r->mask.empty() ? nullptr : r->mask.data();
    d.cross = r->cross.empty() ? nullptr : r->cross.data();
    mol_status ms = molt::plan_create_async(&d, st, &r->plan, s->pool);
    if (ms != MOL_OK) return sfail(ms, mol_last_error());
    if (hipMallocFromPoolAsync(&r->d_prev, r->field, s->pool, st) != hipSuccess ||
        hipMallocFromPoolAsync(&r->d_curr, r->field, s->pool, st) != hipSuccess)
        return sfail(MOL_E_NOMEM, "stream-ordered allocation of the state fields failed");
    if (hipMemcpyAsync(r->d_prev, r->u0, r->field,
                       r->u0_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                       st) != hipSuccess)
        return sfail(MOL_E_DEVICE, "copy of the initial field failed");
    ms = mol_start(r->plan, r->d_prev, nullptr, r->d_curr, st);
    if (ms != MOL_OK) return sfail(ms, mol_last_error());
    mol_plan_ *pl = r->plan;
    if (!pl->solve_step.empty() &&
        molt::run_program(pl, pl->solve_pro, r->d_prev, r->d_curr, nullptr, nullptr, nullptr, st) != hipSuccess)
        return sfail(MOL_E_DEVICE, "launch failed");
    if (hipEventCreateWithFlags(&r->done, hipEventDisableTiming) != hipSuccess)
        return sfail(MOL_E_DEVICE, "completion event failed");
    // argument sets of the step for both buffer roles (masked plans run their
    // launches directly)
    r->direct = pl->masked;
    if (!pl->masked) {
        const molt::Program &prog = pl->solve_step.empty() ? pl->step : pl->solve_step;
        const size_t asz = molt::sweep_args_bytes(pl->fp64);
        for (int par = 0; par < 2 && !r->direct; ++par) {
            void *A = par ? r->d_curr : r->d_prev, *B = par ? r->d_prev : r->d_curr;
            r->args[par].resize(prog.size() * asz);
            for (int k = 0; k < (int)prog.size(); ++k) {
                const void *fp[molt::MAXF];
                void *op[molt::MAXO + 1];
                // three-level step: u_next overwrites u_prev
                molt::resolve_op(pl, prog[k], A, B, A, nullptr, nullptr, fp, op);
                Req::Cached c{k, molt::SweepKey{}, 0, k * asz, asz};
                if (!molt::sweep_prepare(prog[k].op, pl->geom, pl->dc[prog[k].op.dir], pl->fp64, fp, op,
                                         prog[k].cfg, r->args[par].data() + c.off, c.key, c.blocks)) {
                    r->direct = true;
                    break;
                }
                r->ops[par].push_back(c);
            }
        }
    }
    r->left = r->nsteps - 1;
    if (r->left == 0) {
        if (hipEventRecord(r->done, st) != hipSuccess) return sfail(MOL_E_DEVICE, "completion event failed");
        r->recorded = true;
    }
    return MOL_OK;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Batched mode: issue one round (one step of every running request) if a
// staging slot is free.  Returns false when nothing was issued.
bool issue_round(mol_server_ *s)
{
    std::vector<Req *> act;
    for (auto &kv : s->reqs)
        if (kv.second->state == Q_RUNNING && kv.second->left > 0) act.push_back(kv.second);
    if (act.empty()) return false;
    mol_server_::Slot &sl = s->slots[s->rounds % mol_server_::NSLOT];
    if (sl.used && hipEventQuery(sl.ev) == hipErrorNotReady) return false;
    hipStream_t st = s->streams[0];

    struct Ent {
        int64_t blocks;
        const unsigned char *args;    // argument set (cached by the request)
        size_t bytes;
    };
    struct Direct {
        int k;
        Req *r;
        const molt::ProgOp *po;
    };
    std::map<std::pair<int, molt::SweepKey>, std::vector<Ent>> groups;
    std::vector<Direct> direct;
    int maxk = 0;
    for (Req *r : act) {
        mol_plan_ *pl = r->plan;
        const molt::Program &prog = pl->solve_step.empty() ? pl->step : pl->solve_step;
        maxk = std::max(maxk, (int)prog.size());
        if (r->direct) {
            for (int k = 0; k < (int)prog.size(); ++k) direct.push_back({k, r, &prog[k]});
            continue;
        }
        for (const Req::Cached &c : r->ops[r->par])
            groups[{c.k, c.key}].push_back({c.blocks, r->args[r->par].data() + c.off, c.bytes});
    }
    // table layout: per group, first[] (nent + 1) then the argument sets
    size_t total = 0;
    for (auto &g : groups) {
        total += align256((g.second.size() + 1) * sizeof(int64_t));
        for (const Ent &e : g.second) total += e.bytes;
        total = align256(total);
    }
    if (total > sl.cap) {
        if (sl.h) (void)hipHostFree(sl.h);
        if (sl.d) (void)hipFreeAsync(sl.d, st);
        sl.h = sl.d = nullptr;
        sl.cap = 0;
        const size_t cap = std::max(total * 2, (size_t)1 << 20);
        if (hipHostMalloc(&sl.h, cap, hipHostMallocDefault) != hipSuccess ||
            hipMallocFromPoolAsync(&sl.d, cap, s->pool, st) != hipSuccess) {
            s_err = "round table allocation failed";
            for (Req *r : act) {
                r->err = s_err;
                r->state = Q_FAILED;
            }
            return false;
        }
        sl.cap = cap;
    }
    struct Launch {
        int k;
        molt::SweepKey key;
        size_t tab, first;
        int nent;
        int64_t blocks;
    };
    std::vector<Launch> ls;
    unsigned char *h = static_cast<unsigned char *>(sl.h);
    size_t pos = 0;
    for (auto &g : groups) {
        const size_t nent = g.second.size();
        int64_t *first = reinterpret_cast<int64_t *>(h + pos);
        const size_t fpos = pos;
        pos += align256((nent + 1) * sizeof(int64_t));
        const size_t tpos = pos;
        int64_t b = 0;
        for (size_t i = 0; i < nent; ++i) {
            const Ent &e = g.second[i];
            first[i] = b;
            b += e.blocks;
            std::memcpy(h + pos, e.args, e.bytes);
            pos += e.bytes;
        }
        first[nent] = b;
        pos = align256(pos);
        ls.push_back({g.first.first, g.first.second, tpos, fpos, (int)nent, b});
    }
    if (pos > 0 && (hipMemcpyAsync(sl.d, sl.h, pos, hipMemcpyHostToDevice, st) != hipSuccess ||
                    hipEventRecord(sl.ev, st) != hipSuccess)) {
        s_err = "round table copy failed";
        for (Req *r : act) {
            r->err = s_err;
            r->state = Q_FAILED;
        }
        return false;
    }
    if (pos > 0) sl.used = true;
    // launches in step order: position k of every request after position k-1
    hipError_t e = hipSuccess;
    for (int k = 0; k < maxk && e == hipSuccess; ++k) {
        for (const Direct &dr : direct) {
            if (dr.k != k || e != hipSuccess) continue;
            const molt::Program one(1, *dr.po);
            e = molt::run_program(dr.r->plan, one, dr.r->d_prev, dr.r->d_curr, dr.r->d_prev, nullptr,
                                  nullptr, st);
            ++s->launches;
            ++s->sweeps;
        }
        for (const Launch &l : ls) {
            if (l.k != k || e != hipSuccess) continue;
            unsigned char *d = static_cast<unsigned char *>(sl.d);
            e = molt::launch_sweep_batch(l.key, d + l.tab, reinterpret_cast<const int64_t *>(d + l.first),
                                         l.nent, l.blocks, st);
            ++s->launches;
            s->sweeps += l.nent;
        }
    }
    for (Req *r : act) {
        if (e != hipSuccess) {
            r->err = hipGetErrorString(e);
            r->state = Q_FAILED;
            continue;
        }
        std::swap(r->d_prev, r->d_curr);     // the new field is u^n
        r->par ^= 1;
        if (--r->left == 0) {
            if (hipEventRecord(r->done, st) == hipSuccess) r->recorded = true;
            else {
                r->err = "completion event failed";
                r->state = Q_FAILED;
            }
        }
    }
    ++s->rounds;
    return true;
}

// Retire finished requests, then admit from the head of the queue while the
// budget allows.  Appends the ids that finished to done.
void pump(mol_server_ *s, std::vector<int64_t> &done)
{
    for (auto &kv : s->reqs) {
        Req *r = kv.second;
        if (s->batched && r->state == Q_FAILED && r->plan) {
            // failed inside a round: nothing of it may be in flight any more
            (void)hipStreamSynchronize(s->streams[0]);
            retire(s, r);
            ++s->completed;
            done.push_back(r->id);
            continue;
        }
        if (r->state != Q_RUNNING) continue;
        if (s->batched && !r->recorded) continue;
        const hipError_t e = hipEventQuery(r->done);
        if (e == hipErrorNotReady) continue;
        r->state = (e == hipSuccess) ? Q_DONE : Q_FAILED;
        if (e != hipSuccess) r->err = hipGetErrorString(e);
        retire(s, r);
        ++s->completed;
        done.push_back(r->id);
    }
    while (!s->queue.empty()) {
        Req *r = s->queue.front();
        if (s->used + r->footprint > s->budget) break;
        s->queue.pop_front();
        s->used += r->footprint;
        if (s->used > s->peak) s->peak = s->used;
        const double ta = now_s();
        const mol_status ls = s->batched ? admit_batched(s, r) : launch(s, r);
        const double dt = now_s() - ta;
        s->admit_s += dt;
        if (dt > s->admit_max_s) s->admit_max_s = dt;
        if (ls != MOL_OK) {
            r->err = s_err;
            r->state = Q_FAILED;
            // nothing of the request may be in flight any more
            (void)hipStreamSynchronize(s->streams[r->stream]);
            retire(s, r);
            done.push_back(r->id);
            continue;
        }
        r->state = Q_RUNNING;
    }
    if (s->batched) {
        const double tr = now_s();
        while (issue_round(s)) {
        }
        s->round_s += now_s() - tr;
    }
}

}  // namespace

extern "C" {

const char *mol_server_last_error(void) { return s_err.c_str(); }

mol_status mol_server_create(size_t hbm_budget_bytes, int nstreams, mol_server **out)
{
    if (!out || hbm_budget_bytes == 0 || nstreams < 1 || nstreams > 64)
        return sfail(MOL_E_INVALID, "need an out-pointer, a budget > 0 and 1..64 streams");
    mol_server_ *s = new (std::nothrow) mol_server_();
    if (!s) return sfail(MOL_E_NOMEM, "host allocation failed");
    s->budget = hbm_budget_bytes;
    s->t0 = now_s();
    for (int i = 0; i < nstreams; ++i) {
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
            delete s;
            return sfail(MOL_E_DEVICE, "stream creation failed");
        }
        s->streams.push_back(st);
    }
    s->load.assign(s->streams.size(), 0.0);
    if (hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking) != hipSuccess) {
        for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
        delete s;
        return sfail(MOL_E_DEVICE, "stream creation failed");
    }
    int dev = 0;
    (void)hipGetDevice(&dev);
    hipMemPoolProps pp{};
    pp.allocType = hipMemAllocationTypePinned;
    pp.handleTypes = hipMemHandleTypeNone;
    pp.location.type = hipMemLocationTypeDevice;
    pp.location.id = dev;
    uint64_t keep = UINT64_MAX;
    if (hipMemPoolCreate(&s->pool, &pp) != hipSuccess ||
        hipMemPoolSetAttribute(s->pool, hipMemPoolAttrReleaseThreshold, &keep) != hipSuccess) {
        if (s->pool) (void)hipMemPoolDestroy(s->pool);
        for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
        (void)hipStreamDestroy(s->copy);
        delete s;
        return sfail(MOL_E_DEVICE, "memory pool creation failed");
    }
    *out = s;
    return MOL_OK;
}

mol_status mol_server_create_ex(size_t hbm_budget_bytes, int nstreams, int flags, mol_server **out)
{
    if (flags & ~MOL_SERVER_BATCHED) return sfail(MOL_E_INVALID, "unknown server flags");
    mol_status ms = mol_server_create(hbm_budget_bytes, nstreams, out);
    if (ms != MOL_OK || !(flags & MOL_SERVER_BATCHED)) return ms;
    mol_server_ *s = *out;
    s->batched = true;
    for (auto &sl : s->slots) {
        if (hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) != hipSuccess) {
            *out = nullptr;
            (void)mol_server_destroy(s);
            return sfail(MOL_E_DEVICE, "event creation failed");
        }
    }
    return MOL_OK;
}

mol_status mol_server_destroy(mol_server *s)
{
    if (!s) return MOL_OK;
    for (hipStream_t st : s->streams) (void)hipStreamSynchronize(st);
    std::vector<int64_t> done;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        pump(s, done);
        for (auto &kv : s->reqs) {
            Req *r = kv.second;
            if (r->state == Q_RUNNING) retire(s, r);
            if (r->d_curr) (void)hipFreeAsync(r->d_curr, s->copy);
            delete r;
        }
        s->reqs.clear();
    }
    for (hipStream_t st : s->streams) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    for (auto &sl : s->slots) {
        if (sl.h) (void)hipHostFree(sl.h);
        if (sl.d) (void)hipFreeAsync(sl.d, s->copy);
        if (sl.ev) (void)hipEventDestroy(sl.ev);
    }
    (void)hipStreamSynchronize(s->copy);
    (void)hipStreamDestroy(s->copy);
    // every allocation from the pool has been freed and the frees completed
    if (s->pool) (void)hipMemPoolDestroy(s->pool);
    delete s;
    return MOL_OK;
}

mol_status mol_server_submit(mol_server *s, const mol_desc *desc, const void *u0, int u0_on_device,
                             int64_t nsteps, int64_t *id)
{
    if (!s || !desc || !u0 || !id) return sfail(MOL_E_INVALID, "NULL argument");
    if (nsteps < 1) return sfail(MOL_E_INVALID, "nsteps must be >= 1");
    const size_t ws = mol_workspace_bytes(desc);
    if (ws == 0) return sfail(MOL_E_INVALID, std::string("invalid request: ") + mol_last_error());
    Req *r = new (std::nothrow) Req();
    if (!r) return sfail(MOL_E_NOMEM, "host allocation failed");
    r->desc = *desc;
    if (s->batched) r->desc.flags |= MOL_UNIFORM_CONFIG;     // plans of different sizes share kernels
    const int64_t np = npoints(*desc);
    if (desc->mask) r->mask.assign(desc->mask, desc->mask + np);
    if (desc->cross) r->cross.assign(desc->cross, desc->cross + 4 * np);
    r->desc.mask = nullptr;
    r->desc.cross = nullptr;
    r->u0 = u0;
    r->u0_dev = u0_on_device != 0;
    r->nsteps = nsteps;
    r->field = (size_t)np * elem_size(*desc);
    r->footprint = ws + 2 * r->field;
    if (r->footprint > s->budget) {
        delete r;
        return sfail(MOL_E_NOMEM, "request larger than the server's device budget");
    }
    std::vector<int64_t> done;
    std::lock_guard<std::mutex> lk(s->mu);
    r->id = s->next_id++;
    s->reqs[r->id] = r;
    s->queue.push_back(r);
    *id = r->id;
    pump(s, done);     // completions seen here are reported by the next poll
    return MOL_OK;
}

mol_status mol_server_poll(mol_server *s, int64_t *done_ids, int max, int *ndone)
{
    if (!s || !ndone || (max > 0 && !done_ids)) return sfail(MOL_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    std::vector<int64_t> done;
    pump(s, done);
    // every finished request not reported yet (also those seen during submit)
    int n = 0;
    for (auto &kv : s->reqs) {
        Req *r = kv.second;
        if ((r->state == Q_DONE || r->state == Q_FAILED) && !r->reported && n < max) {
            done_ids[n++] = r->id;
            r->reported = true;
        }
    }
    *ndone = n;
    return MOL_OK;
}

mol_status mol_server_result(mol_server *s, int64_t id, void *dst, int dst_on_device)
{
    if (!s || !dst) return sfail(MOL_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return sfail(MOL_E_INVALID, "unknown request id");
    Req *r = it->second;
    if (r->state == Q_QUEUED || r->state == Q_RUNNING) return sfail(MOL_E_INVALID, "request not finished");
    // the request's work is complete (its event fired): copy on the server's
    // copy stream, without waiting for later requests on the request's stream
    hipStream_t st = s->copy;
    mol_status ms = MOL_OK;
    if (r->state == Q_FAILED) {
        ms = sfail(MOL_E_DEVICE, "request failed: " + r->err);
    } else if (hipMemcpyAsync(dst, r->d_curr, r->field,
                              dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                              st) != hipSuccess ||
               hipStreamSynchronize(st) != hipSuccess) {
        ms = sfail(MOL_E_DEVICE, "copy of the result failed");
    }
    if (r->d_curr) (void)hipFreeAsync(r->d_curr, st);
    s->used -= r->field;
    s->reqs.erase(it);
    delete r;
    return ms;
}

mol_status mol_server_stats(mol_server *s, mol_server_info *info)
{
    if (!s || !info) return sfail(MOL_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    std::memset(info, 0, sizeof *info);
    for (auto &kv : s->reqs) {
        if (kv.second->state == Q_QUEUED) ++info->queued;
        else if (kv.second->state == Q_RUNNING) ++info->running;
        else ++info->finished;
    }
    info->completed = s->completed;
    info->bytes_in_use = s->used;
    info->bytes_peak = s->peak;
    info->budget = s->budget;
    info->admit_seconds = s->admit_s;
    info->admit_max_seconds = s->admit_max_s;
    info->round_seconds = s->round_s;
    info->rounds = s->rounds;
    info->launches = s->launches;
    info->sweeps = s->sweeps;
    return MOL_OK;
}

}  // extern "C"
