// Request server: many independent solves of differing size and order served
// concurrently on one GPU.  Requests are admitted in arrival order while their
// device footprint (plan workspace, line-object tables, two state fields) fits
// a byte budget; an admitted request keeps its fields resident in HBM, runs
// start + (nsteps - 1) steps from its own captured hipGraph on one stream of a
// pool (default priority; requests on different streams overlap on the
// hardware queues), and signals completion with an event.  All allocations of
// a request are stream-ordered, so admitting and retiring requests never
// synchronises the device.
#include <hip/hip_runtime.h>

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
    hipStream_t copy = nullptr;       // results leave on their own stream
    int64_t next_id = 1;
    std::deque<Req *> queue;
    std::map<int64_t, Req *> reqs;
    int64_t completed = 0;
    std::mutex mu;
    double t0 = 0;
    double admit_s = 0;               // host time spent admitting requests
    double admit_max_s = 0;
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

// Release everything but the result field.
void retire(mol_server_ *s, Req *r)
{
    hipStream_t st = s->streams[r->stream];
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
    mol_status ms = molt::plan_create_async(&d, st, &r->plan);
    if (ms != MOL_OK) return sfail(ms, mol_last_error());
    if (hipMallocAsync(&r->d_prev, r->field, st) != hipSuccess ||
        hipMallocAsync(&r->d_curr, r->field, st) != hipSuccess)
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

// Retire finished requests, then admit from the head of the queue while the
// budget allows.  Appends the ids that finished to done.
void pump(mol_server_ *s, std::vector<int64_t> &done)
{
    for (auto &kv : s->reqs) {
        Req *r = kv.second;
        if (r->state != Q_RUNNING) continue;
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
        const mol_status ls = launch(s, r);
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
    *out = s;
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
            if (r->d_curr) (void)hipFreeAsync(r->d_curr, s->streams[r->stream]);
            delete r;
        }
        s->reqs.clear();
    }
    for (hipStream_t st : s->streams) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    (void)hipStreamSynchronize(s->copy);
    (void)hipStreamDestroy(s->copy);
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
    return MOL_OK;
}

}  // extern "C"
