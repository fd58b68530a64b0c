// Serving core of libheatst: admission by resident bytes, per-size-class
// batched plans and continuous batching of independent heat solves
// (include/heatst.h, hs_server_*).
//
// Layout of the caller's pool: the shared workspace of every class's plan
// (lane control blocks, tables, partials) at the front, then a heap from
// which each admitted request's fields and multigrid hierarchy are carved
// (first fit, 256-byte blocks, freed blocks coalesce).  A request is
// admitted -- given a lane of its class's plan and its bytes from the heap --
// while the bytes of all admitted requests stay within the budget; the
// class's worker binds the memory to the lane at its next step boundary.
#include "heatst.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <iterator>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

namespace {

struct Request {
    uint64_t ticket;
    int n;
    double nu, dt, t0;
    int nsteps;
    const double* d_u0;
    double* d_out;
    size_t heap_off;
    hs_request_info info;
};

struct Class {
    int idx = 0;
    int n = 0;
    int slots = 0;                         // lanes of the class's plan
    size_t lane_bytes = 0;                 // heap bytes one request of this class holds
    hs_plan* plan = nullptr;
    void* ws = nullptr;                    // the plan's shared workspace
    size_t bytes = 0;
    hipStream_t stream = nullptr;
    std::vector<uint64_t> lane_ticket;     // 0 = free
    std::vector<uint64_t> to_bind;         // admitted, memory not yet bound (lane order of admission)
    std::thread worker;
};

double now_since(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

bool valid_n(int n) { return n >= 1 && n <= 511 && ((n + 1) & n) == 0; }

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

hs_problem class_problem(const hs_server_desc* d, int c)
{
    hs_problem pb;
    std::memset(&pb, 0, sizeof(pb));
    pb.nu = 0.1;
    pb.dt = 0.01;
    pb.t0 = 0.0;
    pb.forcing_c = d->forcing_c;
    pb.nsteps = 0;
    pb.nlevels = 1;
    pb.lev[0].n = d->class_n[c];
    pb.lev[0].order = d->order;
    pb.lev[0].nnodes = d->nnodes;
    pb.mg = d->mg;
    pb.sweeps = d->sweeps;
    pb.sdc_tol = d->sdc_tol;
    pb.max_sweeps = d->max_sweeps;
    pb.batch = d->class_slots[c];
    pb.nslices = 1;
    pb.h_lane_n = nullptr;
    pb.lane_memory = 1;
    return pb;
}

hs_status validate(const hs_server_desc* d)
{
    if (!d || d->nclasses < 1 || d->nclasses > HS_MAX_CLASSES) return HS_EINVAL;
    for (int c = 0; c < d->nclasses; c++) {
        if (!valid_n(d->class_n[c]) || d->class_slots[c] < 1 || d->class_slots[c] > 4096) return HS_EINVAL;
        for (int e = 0; e < c; e++)
            if (d->class_n[e] == d->class_n[c]) return HS_EINVAL;
    }
    return HS_OK;
}

// Shared workspace of every class and the heap bytes of one request per class.
hs_status class_sizes(const hs_server_desc* d, std::vector<size_t>* shared, std::vector<size_t>* lane)
{
    hs_status s = validate(d);
    if (s != HS_OK) return s;
    shared->assign(d->nclasses, 0);
    lane->assign(d->nclasses, 0);
    for (int c = 0; c < d->nclasses; c++) {
        hs_problem pb = class_problem(d, c);
        size_t b = 0;
        if ((s = hs_workspace_bytes(&pb, &b)) != HS_OK) return s;
        (*shared)[c] = align256(b);
        if ((s = hs_lane_bytes(&pb, 0, &b)) != HS_OK) return s;
        (*lane)[c] = align256(b);
    }
    return HS_OK;
}

// First-fit allocator over [0, size) in 256-byte blocks; freed blocks coalesce.
struct Heap {
    std::map<size_t, size_t> free_;   // offset -> length
    void init(size_t size)
    {
        free_.clear();
        if (size >= 256) free_[0] = size & ~(size_t)255;
    }
    bool alloc(size_t bytes, size_t* off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            size_t rest = it->second - bytes;
            size_t next = it->first + bytes;
            free_.erase(it);
            if (rest) free_[next] = rest;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

}  // namespace

struct hs_server {
    hs_server_desc d;
    int device = 0;
    std::chrono::steady_clock::time_point t0;
    std::vector<Class*> classes;
    char* heap_base = nullptr;
    Heap heap;
    size_t budget = 0;                 // most heap bytes admitted requests may hold together
    size_t resident = 0;               // heap bytes of the admitted requests
    std::mutex mu;
    std::condition_variable cv;        // work arrived / stop
    std::condition_variable done_cv;   // a request finished
    std::unordered_map<uint64_t, Request> reqs;
    std::deque<uint64_t> waiting;      // not yet admitted, in arrival order
    uint64_t next_ticket = 1;
    size_t outstanding = 0;
    bool stop = false;
    hs_status worker_error = HS_OK;
};

namespace {

// Admit waiting requests in arrival order (caller holds S->mu).  A request
// needs a free lane of its class and its bytes within the budget and the
// heap.  The oldest request that a free lane exists for but whose bytes do
// not fit reserves them: the requests behind it may only use what is left
// after it, so a large request is not starved by a stream of small ones,
// while small ones still fill the room it cannot use.
void admit_locked(hs_server* S)
{
    if (S->stop) return;
    size_t reserved = 0;
    bool have_reservation = false;
    bool admitted = false;
    for (auto it = S->waiting.begin(); it != S->waiting.end();) {
        Request& r = S->reqs[*it];
        Class& C = *S->classes[r.info.cls];
        int lane = -1;
        for (int l = 0; l < C.slots && lane < 0; l++)
            if (C.lane_ticket[l] == 0) lane = l;
        if (lane < 0) {
            ++it;
            continue;
        }
        size_t off = 0;
        if (S->resident + reserved + C.lane_bytes <= S->budget && S->heap.alloc(C.lane_bytes, &off)) {
            S->resident += C.lane_bytes;
            r.heap_off = off;
            r.info.state = 1;
            r.info.lane = lane;
            r.info.t_admit = now_since(S->t0);
            C.lane_ticket[lane] = r.ticket;
            C.to_bind.push_back(r.ticket);
            it = S->waiting.erase(it);
            admitted = true;
            continue;
        }
        if (!have_reservation) {
            reserved = C.lane_bytes;
            have_reservation = true;
        }
        ++it;
    }
    if (admitted) S->cv.notify_all();
}

void fail_server(hs_server* S, hs_status e)
{
    std::lock_guard<std::mutex> lk(S->mu);
    S->worker_error = e;
    S->stop = true;
    S->cv.notify_all();
    S->done_cv.notify_all();
}

void worker(hs_server* S, Class* Cp)
{
    Class& C = *Cp;
    (void)hipSetDevice(S->device);
    std::vector<hs_lane_stats> st(C.slots);
    while (true) {
        std::vector<Request> bind;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            auto busy = [&]() {
                for (int l = 0; l < C.slots; l++)
                    if (C.lane_ticket[l] != 0) return true;
                return false;
            };
            while (!S->stop && !busy()) S->cv.wait(lk);
            if (S->stop && !busy()) break;
            for (uint64_t tk : C.to_bind) bind.push_back(S->reqs[tk]);
            C.to_bind.clear();
        }
        // new requests join at this step boundary
        hs_status e = HS_OK;
        for (const Request& r : bind) {
            const int l = r.info.lane;
            if (e == HS_OK) e = hs_plan_bind_lane(C.plan, l, S->heap_base + r.heap_off, C.lane_bytes, C.stream);
            if (e == HS_OK) e = hs_set_lane(C.plan, l, r.nu, r.dt, r.t0, r.nsteps, 1, C.stream);
            if (e == HS_OK) e = hs_set_lane_state(C.plan, l, r.d_u0, C.stream);
        }
        if (e == HS_OK) e = hs_step(C.plan, C.stream);
        hs_status se = hs_stats_read(C.plan, st.data(), C.stream);   // synchronises
        if (e == HS_OK && se < 0 && se != HS_ENOCONV && se != HS_ENONFINITE) e = se;
        if (e != HS_OK && e != HS_ENOCONV && e != HS_ENONFINITE) {
            fail_server(S, e);
            break;
        }
        // retire lanes that reached their step count or failed
        for (int l = 0; l < C.slots; l++) {
            Request r;
            {
                std::lock_guard<std::mutex> lk(S->mu);
                uint64_t tk = C.lane_ticket[l];
                if (tk == 0 || S->reqs[tk].info.state != 1) continue;
                bool pending = false;
                for (uint64_t b : C.to_bind) pending |= b == tk;
                if (pending) continue;   // admitted after this step began
                r = S->reqs[tk];
            }
            if (st[l].steps_done < r.nsteps && st[l].status == HS_OK) continue;
            // the result copy and the lane's release must both succeed, else the
            // request finishes with the failure instead of an unwritten output
            hs_lane_stats fin = st[l];
            hs_status ce = hs_get_lane_state(C.plan, l, r.d_out, C.stream);
            hs_status re = hs_set_lane(C.plan, l, 0.1, 0.01, 0.0, 0, 0, C.stream);
            if (hipStreamSynchronize(C.stream) != hipSuccess && ce == HS_OK) ce = HS_EDEVICE;
            if (re == HS_OK) re = hs_plan_unbind_lane(C.plan, l);
            if (ce != HS_OK) fin.status = ce;
            else if (re != HS_OK) fin.status = re;
            std::lock_guard<std::mutex> lk(S->mu);
            Request& q = S->reqs[r.ticket];
            q.info.state = 2;
            q.info.status = fin.status;
            q.info.stats = fin;
            q.info.t_done = now_since(S->t0);
            C.lane_ticket[l] = 0;
            S->heap.release(q.heap_off, C.lane_bytes);
            S->resident -= C.lane_bytes;
            S->outstanding--;
            admit_locked(S);
            S->done_cv.notify_all();
        }
    }
}

}  // namespace

extern "C" {

hs_status hs_server_pool_bytes(const hs_server_desc* d, size_t* shared_bytes, size_t* full_bytes)
{
    std::vector<size_t> shared, lane;
    hs_status s = class_sizes(d, &shared, &lane);
    if (s != HS_OK) return s;
    if (!shared_bytes && !full_bytes) return HS_EINVAL;
    size_t sh = 0, full = 0;
    for (int c = 0; c < d->nclasses; c++) {
        sh += shared[c];
        full += (size_t)d->class_slots[c] * lane[c];
    }
    if (shared_bytes) *shared_bytes = sh;
    if (full_bytes) *full_bytes = sh + full;
    return HS_OK;
}

hs_status hs_server_request_bytes(const hs_server_desc* d, int32_t n, size_t* bytes)
{
    std::vector<size_t> shared, lane;
    hs_status s = class_sizes(d, &shared, &lane);
    if (s != HS_OK) return s;
    if (!bytes) return HS_EINVAL;
    for (int c = 0; c < d->nclasses; c++)
        if (d->class_n[c] == n) {
            *bytes = lane[c];
            return HS_OK;
        }
    return HS_EINVAL;
}

hs_status hs_server_create(const hs_server_desc* d, void* d_pool, size_t pool_bytes, size_t hbm_budget,
                           hs_server** server)
{
    if (!server || !d_pool || ((uintptr_t)d_pool & 255)) return HS_EINVAL;
    std::vector<size_t> shared, lane;
    hs_status s = class_sizes(d, &shared, &lane);
    if (s != HS_OK) return s;
    size_t sh = 0, big = 0;
    for (int c = 0; c < d->nclasses; c++) {
        sh += shared[c];
        big = std::max(big, lane[c]);
    }
    // the pool and the budget must hold the shared part and one request of every class
    if (pool_bytes < sh + big || hbm_budget < sh + big) return HS_ENOMEM;
    hs_server* S = new (std::nothrow) hs_server();
    if (!S) return HS_ENOMEM;
    S->d = *d;
    S->t0 = std::chrono::steady_clock::now();
    if (hipGetDevice(&S->device) != hipSuccess) {
        delete S;
        return HS_EDEVICE;
    }
    char* base = (char*)d_pool;
    size_t off = 0;
    for (int c = 0; c < d->nclasses; c++) {
        Class* C = new Class();
        C->idx = c;
        C->n = d->class_n[c];
        C->slots = d->class_slots[c];
        C->lane_bytes = lane[c];
        C->lane_ticket.assign(C->slots, 0);
        hs_problem pb = class_problem(d, c);
        C->bytes = shared[c];
        C->ws = base + off;
        off += shared[c];
        hs_status e = HS_OK;
        if (hipStreamCreateWithFlags(&C->stream, hipStreamNonBlocking) != hipSuccess) e = HS_EDEVICE;
        if (e == HS_OK) e = hs_plan_create(&pb, &C->plan);
        if (e == HS_OK) e = hs_plan_bind(C->plan, C->ws, C->bytes, C->stream);
        S->classes.push_back(C);
        if (e != HS_OK) {
            hs_server_destroy(S);
            return e;
        }
    }
    S->heap_base = base + off;
    S->heap.init(pool_bytes - off);
    S->budget = hbm_budget - sh;
    for (Class* C : S->classes) C->worker = std::thread(worker, S, C);
    *server = S;
    return HS_OK;
}

hs_status hs_server_submit(hs_server* S, int32_t n, double nu, double dt, double t0, int32_t nsteps,
                           const double* d_u0, double* d_out, uint64_t* ticket)
{
    if (!S || !d_u0 || !d_out || !ticket || !(nu > 0) || !(dt > 0) || nsteps < 0) return HS_EINVAL;
    Class* C = nullptr;
    for (Class* c : S->classes)
        if (c->n == n) C = c;
    if (!C) return HS_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) return S->worker_error != HS_OK ? S->worker_error : HS_ESTATE;
    Request r;
    std::memset(&r.info, 0, sizeof(r.info));
    r.ticket = S->next_ticket++;
    r.n = n;
    r.nu = nu;
    r.dt = dt;
    r.t0 = t0;
    r.nsteps = nsteps;
    r.d_u0 = d_u0;
    r.d_out = d_out;
    r.heap_off = 0;
    r.info.state = 0;
    r.info.cls = C->idx;
    r.info.lane = -1;
    r.info.t_submit = now_since(S->t0);
    S->reqs[r.ticket] = r;
    S->waiting.push_back(r.ticket);
    S->outstanding++;
    *ticket = r.ticket;
    admit_locked(S);
    return HS_OK;
}

hs_status hs_server_poll(hs_server* S, uint64_t ticket, hs_request_info* info)
{
    if (!S) return HS_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return HS_EINVAL;
    if (info) *info = it->second.info;
    if (S->worker_error != HS_OK) return S->worker_error;
    return it->second.info.state == 2 ? HS_OK : HS_PENDING;
}

hs_status hs_server_resident(hs_server* S, size_t* resident_bytes, size_t* budget_bytes)
{
    if (!S) return HS_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    if (resident_bytes) *resident_bytes = S->resident;
    if (budget_bytes) *budget_bytes = S->budget;
    return HS_OK;
}

hs_status hs_server_drain(hs_server* S)
{
    if (!S) return HS_EINVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    while (S->outstanding > 0 && S->worker_error == HS_OK) S->done_cv.wait(lk);
    return S->worker_error;
}

hs_status hs_server_destroy(hs_server* S)
{
    if (!S) return HS_EINVAL;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        S->cv.notify_all();
    }
    for (Class* C : S->classes) {
        if (C->worker.joinable()) C->worker.join();
        if (C->plan) hs_plan_destroy(C->plan);
        if (C->stream) (void)hipStreamDestroy(C->stream);
        delete C;
    }
    delete S;
    return HS_OK;
}

}  // extern "C"
