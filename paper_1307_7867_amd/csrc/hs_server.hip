// Serving core of libheatst: admission, slot management and continuous
// batching of independent heat solves (include/heatst.h, hs_server_*).
#include "heatst.h"

#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
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
    hs_request_info info;
};

struct Class {
    int idx = 0;
    int n = 0;
    int slots = 0;
    hs_plan* plan = nullptr;
    void* ws = nullptr;
    size_t bytes = 0;
    hipStream_t stream = nullptr;
    std::vector<uint64_t> lane_ticket;     // 0 = free
    std::deque<uint64_t> waiting;
    std::thread worker;
};

double now_since(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

bool valid_n(int n) { return n >= 1 && n <= 511 && ((n + 1) & n) == 0; }

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
    return pb;
}

hs_status validate(const hs_server_desc* d)
{
    if (!d || d->nclasses < 1 || d->nclasses > HS_MAX_CLASSES) return HS_EINVAL;
    for (int c = 0; c < d->nclasses; c++) {
        if (!valid_n(d->class_n[c]) || d->class_slots[c] < 1) return HS_EINVAL;
        for (int e = 0; e < c; e++)
            if (d->class_n[e] == d->class_n[c]) return HS_EINVAL;
    }
    return HS_OK;
}

}  // namespace

struct hs_server {
    hs_server_desc d;
    int device = 0;
    std::chrono::steady_clock::time_point t0;
    std::vector<Class*> classes;
    std::mutex mu;
    std::condition_variable cv;        // work arrived / stop
    std::condition_variable done_cv;   // a request finished
    std::unordered_map<uint64_t, Request> reqs;
    uint64_t next_ticket = 1;
    size_t outstanding = 0;
    bool stop = false;
    hs_status worker_error = HS_OK;
};

namespace {

void retire(hs_server* S, Class& C, int lane, const hs_lane_stats& st)
{
    uint64_t tk = C.lane_ticket[lane];
    std::lock_guard<std::mutex> lk(S->mu);
    Request& r = S->reqs[tk];
    r.info.state = 2;
    r.info.status = st.status;
    r.info.stats = st;
    r.info.t_done = now_since(S->t0);
    C.lane_ticket[lane] = 0;
    S->outstanding--;
    S->done_cv.notify_all();
}

void worker(hs_server* S, Class* Cp)
{
    Class& C = *Cp;
    (void)hipSetDevice(S->device);
    std::vector<hs_lane_stats> st(C.slots);
    while (true) {
        std::vector<std::pair<int, Request>> admitted;
        int active = 0;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            for (int l = 0; l < C.slots; l++) active += C.lane_ticket[l] != 0;
            while (!S->stop && active == 0 && C.waiting.empty()) {
                S->cv.wait(lk);
            }
            if (S->stop && active == 0 && C.waiting.empty()) break;
            for (int l = 0; l < C.slots && !C.waiting.empty(); l++) {
                if (C.lane_ticket[l] != 0) continue;
                uint64_t tk = C.waiting.front();
                C.waiting.pop_front();
                C.lane_ticket[l] = tk;
                Request& r = S->reqs[tk];
                r.info.state = 1;
                r.info.lane = l;
                r.info.t_admit = now_since(S->t0);
                admitted.push_back({l, r});
                active++;
            }
        }
        hs_status e = HS_OK;
        for (auto& a : admitted) {
            const Request& r = a.second;
            if (e == HS_OK) e = hs_set_lane(C.plan, a.first, r.nu, r.dt, r.t0, r.nsteps, 1, C.stream);
            if (e == HS_OK) e = hs_set_lane_state(C.plan, a.first, r.d_u0, C.stream);
        }
        if (e == HS_OK) e = hs_step(C.plan, C.stream);
        hs_status se = hs_stats_read(C.plan, st.data(), C.stream);   // synchronises
        if (e == HS_OK && se < 0 && se != HS_ENOCONV && se != HS_ENONFINITE) e = se;
        if (e != HS_OK && e != HS_ENOCONV && e != HS_ENONFINITE) {
            std::lock_guard<std::mutex> lk(S->mu);
            S->worker_error = e;
            S->stop = true;
            S->cv.notify_all();
            S->done_cv.notify_all();
            break;
        }
        // retire lanes that reached their step count or failed
        for (int l = 0; l < C.slots; l++) {
            uint64_t tk = C.lane_ticket[l];
            if (tk == 0) continue;
            int nsteps;
            double* out;
            {
                std::lock_guard<std::mutex> lk(S->mu);
                nsteps = S->reqs[tk].nsteps;
                out = S->reqs[tk].d_out;
            }
            if (st[l].steps_done < nsteps && st[l].status == HS_OK) continue;
            // the result copy and the lane's release must both succeed, else the
            // request finishes with the failure instead of an unwritten output
            hs_lane_stats fin = st[l];
            hs_status ce = hs_get_lane_state(C.plan, l, out, C.stream);
            hs_status re = hs_set_lane(C.plan, l, 0.1, 0.01, 0.0, 0, 0, C.stream);
            if (hipStreamSynchronize(C.stream) != hipSuccess && ce == HS_OK) ce = HS_EDEVICE;
            if (ce != HS_OK) fin.status = ce;
            else if (re != HS_OK) fin.status = re;
            retire(S, C, l, fin);
        }
    }
}

}  // namespace

extern "C" {

hs_status hs_server_pool_bytes(const hs_server_desc* d, size_t* bytes)
{
    hs_status s = validate(d);
    if (s != HS_OK) return s;
    if (!bytes) return HS_EINVAL;
    size_t total = 0;
    for (int c = 0; c < d->nclasses; c++) {
        hs_problem pb = class_problem(d, c);
        size_t b = 0;
        s = hs_workspace_bytes(&pb, &b);
        if (s != HS_OK) return s;
        total += (b + 255) & ~(size_t)255;
    }
    *bytes = total;
    return HS_OK;
}

hs_status hs_server_create(const hs_server_desc* d, void* d_pool, size_t pool_bytes, size_t hbm_budget,
                           hs_server** server)
{
    if (!server || !d_pool || ((uintptr_t)d_pool & 255)) return HS_EINVAL;
    size_t need = 0;
    hs_status s = hs_server_pool_bytes(d, &need);
    if (s != HS_OK) return s;
    if (need > pool_bytes || need > hbm_budget) return HS_ENOMEM;
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
        C->lane_ticket.assign(C->slots, 0);
        hs_problem pb = class_problem(d, c);
        hs_workspace_bytes(&pb, &C->bytes);
        C->ws = base + off;
        off += (C->bytes + 255) & ~(size_t)255;
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
    r.info.state = 0;
    r.info.cls = C->idx;
    r.info.lane = -1;
    r.info.t_submit = now_since(S->t0);
    S->reqs[r.ticket] = r;
    C->waiting.push_back(r.ticket);
    S->outstanding++;
    *ticket = r.ticket;
    S->cv.notify_all();
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
