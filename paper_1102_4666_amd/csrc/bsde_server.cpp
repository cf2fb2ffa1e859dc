// bsde_server.cpp -- continuous-batching request server of libbsde.so.
//
// Requests (a pricing problem plus a query point) are admitted while their
// device footprint fits the server's HBM budget and the number in flight is
// below the limit.  Set-up threads build admitted problems (host set-up and
// upload) while the GPU works on others.  Two engine lanes, each a thread
// with a stream of its own, advance the in-flight problems with the batched
// persistent kernels: the light lane the problems whose Picard iteration is
// cheap (a few milliseconds of GPU time), the heavy lane the others, so
// that a cheap request never waits for a step of the heaviest problems;
// their launches share the GPU.  In each lane, problems that arrive while
// others are on the GPU join at the next step, finished ones leave,
// release their memory and complete their tickets.  Each problem keeps its coefficients and channel tables
// resident on the device across iterations.  A problem's result does not
// depend on what else is in flight: its tiles and reductions are those of a
// solve alone.
#include "bsde_internal.h"

#include <algorithm>
#include <cmath>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>

using namespace bsde;
using Clock = std::chrono::steady_clock;

namespace {
double ms_between(Clock::time_point a, Clock::time_point b)
{
    return std::chrono::duration<double, std::milli>(b - a).count();
}

struct Request {
    unsigned long long ticket = 0;
    int d = 0;
    std::vector<double> level, div, S0, qS;
    bsde_sigma sigma{};
    bsde_payoff payoff{};
    bsde_grid grid{};
    double r = 0;
    int M = 0, N = 0, K_it = 0, precision = 0;
    double penalty = 0, qt = 0;
    unsigned long long seed = 0;
    size_t bytes = 0;
    double path_steps = 0;
    bsde_problem h = nullptr;
    Clock::time_point t_submit, t_start, t_done;
    bool done = false;
    bsde_result result{};
};
} // namespace

// One engine lane: its thread and stream, the problems built for it and
// not yet joined, and those it advances.
struct EngineLane {
    hipStream_t stream = nullptr;
    std::condition_variable cv;
    std::deque<Request *> ready;
    std::vector<Request *> active;
    std::thread thread;
};
constexpr int kLight = 0, kHeavy = 1, kLanes = 2;

struct bsde_server_s {
    size_t budget = 0, reserved = 0;
    int max_inflight = 0, inflight = 0; // inflight: in set-up, ready or active
    int device = 0;
    std::mutex mu;
    std::condition_variable cv_admit, cv_done;
    std::deque<Request *> pending;
    EngineLane lanes[kLanes];
    std::map<unsigned long long, Request *> tickets;
    unsigned long long next_ticket = 1;
    bool stop = false;
    std::vector<std::thread> setup_threads;
    // statistics
    std::vector<double> latencies;
    double steps_done = 0;
    long completed = 0, engine_steps = 0;
    Clock::time_point t_first, t_last;
    bool any = false;
};

static void complete(bsde_server_s *S, Request *q, int status)
{
    q->t_done = Clock::now();
    q->result.status = status;
    q->result.latency_ms = ms_between(q->t_submit, q->t_done);
    q->result.queue_ms = ms_between(q->t_submit, q->t_start);
    q->done = true;
    if (status == BSDE_OK) {
        S->latencies.push_back(q->result.latency_ms);
        S->steps_done += q->path_steps;
        S->completed += 1;
        S->t_last = q->t_done;
    }
}

// Relative GPU cost of one Picard iteration of a problem: its path-steps
// over the path-kernel rate of its dimension (path-steps/s measured on
// MI355X with FP32 paths at the benchmark workloads; FP64 paths are 3-4x
// slower).  Used only to group iterations into engine steps and problems
// into the light and heavy lanes.
static double iteration_cost(const bsde_problem_s *h)
{
    double rate = h->d <= 1 ? 1.6e12 : h->d <= 2 ? 7e11 : h->d <= 3 ? 5e11
                : h->d <= 5 ? 3e11 : 1.1e11;
    if (h->precision != BSDE_FP32_PATHS) rate /= 3.5;
    return (double)h->n * h->M * h->N / rate + 2e-5; // + launch overheads
}

// problems whose iteration costs less than this go to the light lane
static constexpr double kLightIteration = 5e-3; // seconds
// compute units whose workgroup slots the heavy lane's grids leave free
static constexpr int kLightCUs = 16;

static void setup_loop(bsde_server_s *S)
{
    (void)hipSetDevice(S->device);
    for (;;) {
        Request *q = nullptr;
        {
            std::unique_lock<std::mutex> g(S->mu);
            S->cv_admit.wait(g, [&] {
                if (S->stop) return true;
                if (S->pending.empty() || S->inflight >= S->max_inflight) return false;
                const size_t b = S->pending.front()->bytes;
                // admit when it fits; a request larger than the whole budget
                // is admitted alone
                return S->reserved + b <= S->budget || S->reserved == 0;
            });
            if (S->stop) return;
            q = S->pending.front();
            S->pending.pop_front();
            S->reserved += q->bytes;
            S->inflight += 1;
            q->t_start = Clock::now();
        }
        bsde_problem h = nullptr;
        bsde_status st = bsde_create_problem(q->d, &q->sigma, q->r, &q->payoff, &q->grid,
                                             q->M, q->N, q->K_it, q->penalty, q->seed,
                                             q->precision, &h);
        std::lock_guard<std::mutex> g(S->mu);
        if (st != BSDE_OK) {
            S->reserved -= q->bytes;
            S->inflight -= 1;
            complete(S, q, st);
            S->cv_done.notify_all();
            S->cv_admit.notify_all();
            continue;
        }
        q->h = h;
        EngineLane &L = S->lanes[iteration_cost(h) < kLightIteration ? kLight : kHeavy];
        L.ready.push_back(q);
        L.cv.notify_one();
    }
}

static void finish(bsde_server_s *S, Request *q)
{
    // coefficients back, price and deltas at the query point, release
    int status = fetch_coefficients(q->h);
    if (status == BSDE_OK) {
        double price = 0, delta[kMaxD] = {0};
        status = bsde_query_price_delta(q->h, 1, &q->qt, q->qS.data(), &price, delta);
        q->result.price = price;
        for (int j = 0; j < q->d; ++j) q->result.delta[j] = delta[j];
    }
    bsde_destroy(q->h);
    q->h = nullptr;
    std::lock_guard<std::mutex> g(S->mu);
    S->reserved -= q->bytes;
    S->inflight -= 1;
    complete(S, q, status);
    S->cv_done.notify_all();
    S->cv_admit.notify_all();
}

// most iterations of one problem chained into one engine step
static constexpr int kMaxChain = 16;

static void engine_loop(bsde_server_s *S, int lane)
{
    (void)hipSetDevice(S->device);
    EngineLane &L = S->lanes[lane];
    for (;;) {
        {
            std::unique_lock<std::mutex> g(S->mu);
            L.cv.wait(g, [&] {
                return S->stop || !L.ready.empty() || !L.active.empty();
            });
            if (S->stop && L.ready.empty() && L.active.empty()) return;
            while (!L.ready.empty()) { // continuous batching: join now
                L.active.push_back(L.ready.front());
                L.ready.pop_front();
            }
        }
        // One engine step lasts about one iteration of its most expensive
        // problem; cheaper problems run as many of their own iterations in
        // that time (chained in the same batched schedule), so a small
        // request does not wait one heavy iteration per iteration of its
        // own.  Results do not depend on this grouping.
        std::vector<bsde_problem> hs;
        std::vector<double> cost;
        double quantum = 0.0;
        for (Request *q : L.active) {
            hs.push_back(q->h);
            cost.push_back(iteration_cost(q->h));
            quantum = std::max(quantum, cost.back());
        }
        std::vector<int> steps(hs.size());
        for (size_t j = 0; j < hs.size(); ++j)
            steps[j] = (int)std::max(1.0, std::min((double)kMaxChain,
                                                   std::floor(quantum / cost[j])));
        // the heavy lane's signatures run as parallel branches on the
        // library's side streams, and its persistent grids leave the slots
        // of kLightCUs compute units free, so that the light lane's
        // workgroups find room beside them instead of waiting for the
        // heavy kernels to drain; the light lane's small launches stay on
        // its own stream
        bsde_status st = run_batch(hs.data(), (int)hs.size(), L.stream, 1, false, false,
                                   nullptr, steps.data(), nullptr, 0, lane == kHeavy,
                                   lane == kHeavy ? kLightCUs : 0);
        {
            // engine_steps is read by bsde_server_stats under the mutex
            std::lock_guard<std::mutex> g(S->mu);
            S->engine_steps += 1;
        }
        // a request's result is read only after complete() marks it done
        // under the mutex, after these writes
        for (Request *q : L.active) q->result.engine_steps += 1;
        std::vector<Request *> still;
        for (Request *q : L.active) {
            if (st != BSDE_OK) {
                bsde_destroy(q->h);
                q->h = nullptr;
                std::lock_guard<std::mutex> g(S->mu);
                S->reserved -= q->bytes;
                S->inflight -= 1;
                complete(S, q, st);
                S->cv_done.notify_all();
                S->cv_admit.notify_all();
            } else if (q->h->k_done >= q->h->K_it) {
                finish(S, q);
            } else {
                still.push_back(q);
            }
        }
        L.active.swap(still);
    }
}

extern "C" {

bsde_status bsde_server_create(size_t hbm_budget_bytes, int max_inflight,
                               int setup_threads, bsde_server *out)
{
    if (out) *out = nullptr;
    if (!out || hbm_budget_bytes == 0 || max_inflight < 1 || setup_threads < 0 ||
        setup_threads > 64)
        return fail(BSDE_EINVAL, "bad server arguments");
    auto *S = new (std::nothrow) bsde_server_s();
    if (!S) return fail(BSDE_ENOMEM, "host allocation");
    S->budget = hbm_budget_bytes;
    S->max_inflight = max_inflight;
    hipError_t e = hipGetDevice(&S->device);
    for (int l = 0; l < kLanes && e == hipSuccess; ++l)
        e = hipStreamCreateWithFlags(&S->lanes[l].stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        for (int l = 0; l < kLanes; ++l)
            if (S->lanes[l].stream) (void)hipStreamDestroy(S->lanes[l].stream);
        delete S;
        return fail(BSDE_EDEVICE, std::string("server stream: ") + hipGetErrorString(e));
    }
    const int nthreads = setup_threads > 0 ? setup_threads : 4;
    for (int t = 0; t < nthreads; ++t) S->setup_threads.emplace_back(setup_loop, S);
    for (int l = 0; l < kLanes; ++l) S->lanes[l].thread = std::thread(engine_loop, S, l);
    *out = S;
    return BSDE_OK;
}

bsde_status bsde_server_submit(bsde_server S, const bsde_request *req,
                               unsigned long long *ticket)
{
    if (!S || !req || !ticket || !req->sigma.level || !req->payoff.S0)
        return fail(BSDE_EINVAL, "null argument");
    const int d = req->d;
    if (d < 1 || d > kMaxD) return fail(BSDE_EINVAL, "d must be in [1, 10]");
    if (req->grid.redraw)
        return fail(BSDE_EUNSUPPORTED, "points redrawn every iteration are not served");
    if (req->grid.kernel_bw != 0.0)
        return fail(BSDE_EUNSUPPORTED, "the kernel operator is not served");
    auto *q = new (std::nothrow) Request();
    if (!q) return fail(BSDE_ENOMEM, "host allocation");
    q->d = d;
    q->level.assign(req->sigma.level, req->sigma.level + d);
    q->div.assign(d, 0.0);
    if (req->sigma.dividend) q->div.assign(req->sigma.dividend, req->sigma.dividend + d);
    q->S0.assign(req->payoff.S0, req->payoff.S0 + d);
    q->qS = req->query_S ? std::vector<double>(req->query_S, req->query_S + d) : q->S0;
    q->sigma = req->sigma;
    q->sigma.level = q->level.data();
    q->sigma.dividend = q->div.data();
    q->payoff = req->payoff;
    q->payoff.S0 = q->S0.data();
    q->grid = req->grid;
    q->r = req->r;
    q->M = req->M;
    q->N = req->N;
    q->K_it = req->n_picard;
    q->precision = req->precision;
    q->penalty = req->penalty;
    q->qt = req->query_t;
    q->seed = req->seed;
    q->bytes = problem_device_bytes(d, &req->grid, req->M, req->n_picard);
    size_t ns = 1;
    if (req->grid.kind == BSDE_GRID_TENSOR)
        for (int j = 0; j < d; ++j) ns *= (size_t)std::max(1, req->grid.n_x);
    else
        ns = (size_t)std::max(1, req->grid.n_x);
    q->path_steps = (double)ns * req->grid.n_t * req->M * req->N * req->n_picard;
    q->t_submit = Clock::now();
    std::lock_guard<std::mutex> g(S->mu);
    if (S->stop) {
        delete q;
        return fail(BSDE_ESTATE, "server is shutting down");
    }
    q->ticket = S->next_ticket++;
    if (!S->any) {
        S->any = true;
        S->t_first = q->t_submit;
    }
    S->tickets[q->ticket] = q;
    if (q->bytes == 0) { // unsupported (d, eta): fail the ticket at once
        q->t_start = q->t_submit;
        complete(S, q, BSDE_EUNSUPPORTED);
        S->cv_done.notify_all();
    } else {
        S->pending.push_back(q);
        S->cv_admit.notify_one();
    }
    *ticket = q->ticket;
    return BSDE_OK;
}

bsde_status bsde_server_poll(bsde_server S, unsigned long long ticket, int wait,
                             bsde_result *out)
{
    if (!S || !out) return fail(BSDE_EINVAL, "null argument");
    std::unique_lock<std::mutex> g(S->mu);
    auto it = S->tickets.find(ticket);
    if (it == S->tickets.end()) return fail(BSDE_EINVAL, "unknown ticket");
    Request *q = it->second;
    if (!q->done) {
        if (!wait) return fail(BSDE_EBUSY, "request still running");
        S->cv_done.wait(g, [&] { return q->done; });
    }
    *out = q->result;
    S->tickets.erase(it);
    delete q;
    return BSDE_OK;
}

bsde_status bsde_server_stats(bsde_server S, bsde_server_stats_t *st)
{
    if (!S || !st) return fail(BSDE_EINVAL, "null argument");
    std::lock_guard<std::mutex> g(S->mu);
    std::memset(st, 0, sizeof(*st));
    st->completed = S->completed;
    st->engine_steps = S->engine_steps;
    st->in_flight = S->inflight;
    st->pending = (long)S->pending.size();
    st->reserved_bytes = S->reserved;
    if (!S->latencies.empty()) {
        std::vector<double> l = S->latencies;
        std::sort(l.begin(), l.end());
        auto pct = [&](double f) {
            const double pos = f * (l.size() - 1);
            const size_t lo = (size_t)pos;
            const size_t hi = std::min(lo + 1, l.size() - 1);
            return l[lo] + (pos - lo) * (l[hi] - l[lo]);
        };
        st->p50_ms = pct(0.50);
        st->p99_ms = pct(0.99);
        const double span = ms_between(S->t_first, S->t_last) * 1e-3;
        if (span > 0) {
            st->requests_per_s = S->completed / span;
            st->path_steps_per_s = S->steps_done / span;
        }
    }
    return BSDE_OK;
}

void bsde_server_destroy(bsde_server S)
{
    if (!S) return;
    {
        std::lock_guard<std::mutex> g(S->mu);
        S->stop = true;
    }
    S->cv_admit.notify_all();
    for (auto &t : S->setup_threads) t.join();
    // the engines finish what is in flight, then stop
    for (int l = 0; l < kLanes; ++l) {
        {
            std::lock_guard<std::mutex> g(S->mu);
            S->lanes[l].cv.notify_all();
        }
        S->lanes[l].thread.join();
    }
    for (int l = 0; l < kLanes; ++l)
        for (Request *q : S->lanes[l].ready) {
            bsde_destroy(q->h);
            delete q;
        }
    for (Request *q : S->pending) delete q;
    for (auto &kv : S->tickets)
        if (kv.second->done) delete kv.second;
    for (int l = 0; l < kLanes; ++l) (void)hipStreamDestroy(S->lanes[l].stream);
    delete S;
}

} // extern "C"
