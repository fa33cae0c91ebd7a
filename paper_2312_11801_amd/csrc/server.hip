// Request loop for many SDP solves on one GPU (continuous batching).
//
// Requests (an SDP instance, optionally followed by a grown version of it that is
// warm-started from the first solve's state, as in the incremental setting of
// Sec. 5.1) enter a queue.  A fixed set of slots, each a host worker thread with
// its own HIP stream, takes queued requests whenever its slot is free and the
// request's device footprint fits in the remaining HBM budget (first fit in
// arrival order).  Work of different slots is enqueued on different streams and
// overlaps on the device; every instance keeps y, the bundle (V, Xbar scalars,
// zbar) and the sketch resident in its handle between the base solve and the
// warm restart.  Each request's computation depends only on its own data and the
// kernels are deterministic, so a result does not depend on what else runs.
//
// Packed mode replaces the slot threads by one scheduler thread: every admitted
// instance is one workgroup of the packed launches (one launch advances all of them
// by a few iterations of Alg. 1); between launches the scheduler retires finished
// solves, prepares the warm restarts of grown instances and admits queued requests.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/usbs.h"
#include "packed_host.h"

namespace {

// owning copy of a usbs_problem (the caller may free its arrays after submit)
struct OwnedProblem {
    int64_t n = 0, m = 0, nt = 0;
    std::vector<int64_t> rowptr;
    std::vector<int32_t> col, a_row, a_i, a_j;
    std::vector<double> val, a_v, b;
    std::vector<uint8_t> ineq;
    std::vector<float> psi;
    double trace = 0.0;

    void copy_from(const usbs_problem *p, int r) {
        n = p->n;
        m = p->m;
        nt = p->n_triplets;
        trace = p->trace;
        rowptr.assign(p->rowptr, p->rowptr + n + 1);
        const int64_t nnz = rowptr[n];
        col.assign(p->col, p->col + nnz);
        val.assign(p->val, p->val + nnz);
        a_row.assign(p->a_row, p->a_row + nt);
        a_i.assign(p->a_i, p->a_i + nt);
        a_j.assign(p->a_j, p->a_j + nt);
        a_v.assign(p->a_v, p->a_v + nt);
        b.assign(p->b, p->b + m);
        ineq.assign(p->is_ineq, p->is_ineq + m);
        if (p->psi && r > 0) psi.assign(p->psi, p->psi + (size_t)n * r);
    }
    usbs_problem view() const {
        usbs_problem p{};
        p.n = n;
        p.rowptr = rowptr.data();
        p.col = col.data();
        p.val = val.data();
        p.m = m;
        p.n_triplets = nt;
        p.a_row = a_row.data();
        p.a_i = a_i.data();
        p.a_j = a_j.data();
        p.a_v = a_v.data();
        p.b = b.data();
        p.is_ineq = ineq.data();
        p.trace = trace;
        p.psi = psi.empty() ? nullptr : psi.data();
        return p;
    }
};

struct Request {
    int64_t id = 0;
    OwnedProblem base, grown;
    bool has_grown = false;
    int64_t footprint = 0;
    int64_t nmax = 0;   // vertices of the larger of the two instances (packed-mode routing)
    double t_submit = 0.0, t_admit = 0.0, t_base_done = 0.0, t_done = 0.0;
    usbs_result res_base{}, res_grown{};
    int status_base = 0, status_grown = 0;
    int slot = -1;
    bool done = false;
    std::string err;
};

}  // namespace

struct usbs_server {
    usbs_server_config cfg{};
    int dev = 0;
    std::chrono::steady_clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> queue;
    std::map<int64_t, std::unique_ptr<Request>> reqs;
    int64_t next_id = 1;
    int64_t budget = 0, used = 0, peak_used = 0;
    int running = 0, peak_running = 0;
    int64_t completed = 0;
    bool stop = false;
    bool packed = false;      // packed mode: small requests go to the packed launches
    int64_t packed_max_n = 0; // larger requests go to the per-instance workers
    std::vector<std::thread> workers;
    std::string err;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

// which requests a consumer takes: the per-instance workers take all of them in streams mode
// and the large ones in packed mode; the packed scheduler takes the rest
bool eligible(const usbs_server *sv, const Request *rq, bool packed_consumer) {
    if (!sv->packed) return !packed_consumer;
    return packed_consumer == (rq->nmax <= sv->packed_max_n);
}
bool any_eligible(const usbs_server *sv, bool packed_consumer, bool must_fit) {
    for (const Request *q : sv->queue)
        if (eligible(sv, q, packed_consumer) && (!must_fit || sv->used + q->footprint <= sv->budget)) return true;
    return false;
}

void worker(usbs_server *sv, int slot) {
    (void)hipSetDevice(sv->dev);
    hipStream_t stream = nullptr;
    // default priority on purpose: every stream of the library runs at the same priority
    if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess) stream = nullptr;
    for (;;) {
        Request *rq = nullptr;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            // wake when a queued request of this worker fits, or to exit once stopping with
            // none of its requests queued
            sv->cv_work.wait(lk, [&] {
                if (sv->stop && !any_eligible(sv, false, false)) return true;
                return any_eligible(sv, false, true);
            });
            if (sv->stop && !any_eligible(sv, false, false)) break;
            // first fit in arrival order
            for (auto it = sv->queue.begin(); it != sv->queue.end(); ++it)
                if (eligible(sv, *it, false) && sv->used + (*it)->footprint <= sv->budget) {
                    rq = *it;
                    sv->queue.erase(it);
                    break;
                }
            if (!rq) continue;
            sv->used += rq->footprint;
            sv->peak_used = std::max(sv->peak_used, sv->used);
            sv->running++;
            sv->peak_running = std::max(sv->peak_running, sv->running);
            rq->t_admit = sv->now();
            rq->slot = slot;
        }
        usbs_params prm = sv->cfg.params;
        prm.stream = stream;
        usbs_handle *h = nullptr;
        usbs_problem pb = rq->base.view();
        int st = usbs_create(&pb, &prm, &h);
        if (st == USBS_OK) st = usbs_solve(h, &rq->res_base, nullptr, nullptr, nullptr);
        rq->status_base = st;
        rq->t_base_done = sv->now();
        if (st >= 0 && rq->has_grown) {
            // warm restart of the grown instance from the resident state (Sec. 5.1)
            usbs_problem pg = rq->grown.view();
            int st2 = usbs_warm_start(h, &pg);
            if (st2 == USBS_OK) st2 = usbs_solve(h, &rq->res_grown, nullptr, nullptr, nullptr);
            rq->status_grown = st2;
        }
        if ((st < 0 || rq->status_grown < 0) && h) rq->err = usbs_last_error(h);
        usbs_free(h);
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            rq->t_done = sv->now();
            rq->done = true;
            sv->used -= rq->footprint;
            sv->running--;
            sv->completed++;
        }
        sv->cv_done.notify_all();
        sv->cv_work.notify_all();
    }
    if (stream) (void)hipStreamDestroy(stream);
}


// ---------------------------------------------------------------------------
// packed mode: one scheduler thread, one workgroup per admitted instance
// ---------------------------------------------------------------------------
struct Active {
    Request *rq = nullptr;
    usbs_handle *h = nullptr;
    usbs::PackState st{};
    bool grown = false;     // solving the grown instance (after the warm restart)
    double t_phase = 0.0;   // start of the current solve (time limit)
};

void finish_request(usbs_server *sv, Active &a) {
    if (a.h && (a.rq->status_base < 0 || a.rq->status_grown < 0)) a.rq->err = usbs_last_error(a.h);
    usbs_free(a.h);
    a.h = nullptr;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        a.rq->t_done = sv->now();
        a.rq->done = true;
        sv->used -= a.rq->footprint;
        sv->running--;
        sv->completed++;
    }
    sv->cv_done.notify_all();
}

void packer(usbs_server *sv) {
    (void)hipSetDevice(sv->dev);
    // default priority on purpose: every stream of the library runs at the same priority
    hipStream_t launch_stream = nullptr, side_stream = nullptr;
    if (hipStreamCreateWithFlags(&launch_stream, hipStreamNonBlocking) != hipSuccess) launch_stream = nullptr;
    if (hipStreamCreateWithFlags(&side_stream, hipStreamNonBlocking) != hipSuccess) side_stream = nullptr;
    const int iters = sv->cfg.iters_per_launch > 0 ? sv->cfg.iters_per_launch : 8;
    {
        usbs_pack::Runner R(launch_stream);
        std::vector<Active> act;
        for (;;) {
            // admission: first fit in arrival order while a slot is free
            std::vector<Request *> admit;
            {
                std::unique_lock<std::mutex> lk(sv->mu);
                if (act.empty())
                    sv->cv_work.wait(lk, [&] { return sv->stop || any_eligible(sv, true, true); });
                if (act.empty() && sv->stop && !any_eligible(sv, true, false)) break;
                for (auto it = sv->queue.begin(); it != sv->queue.end() && (int)(act.size() + admit.size()) < sv->cfg.slots;) {
                    if (eligible(sv, *it, true) && sv->used + (*it)->footprint <= sv->budget) {
                        Request *rq = *it;
                        it = sv->queue.erase(it);
                        sv->used += rq->footprint;
                        sv->peak_used = std::max(sv->peak_used, sv->used);
                        sv->running++;
                        sv->peak_running = std::max(sv->peak_running, sv->running);
                        rq->t_admit = sv->now();
                        admit.push_back(rq);
                    } else {
                        ++it;
                    }
                }
            }
            for (Request *rq : admit) {
                usbs_params prm = sv->cfg.params;
                prm.stream = side_stream;
                prm.autotune = 0;   // the packed kernel has one launch shape
                Active a;
                a.rq = rq;
                a.t_phase = sv->now();
                usbs_problem pb = rq->base.view();
                const int st = usbs_pack::create(&pb, &prm, &a.h, false);
                rq->slot = -1;
                if (st != USBS_OK) {
                    rq->status_base = st;
                    rq->t_base_done = sv->now();
                    finish_request(sv, a);
                    continue;
                }
                a.st = usbs_pack::begin(a.h, usbs::PACK_INIT_COLD);
                act.push_back(a);
            }
            if (act.empty()) continue;
            // one packed launch over every active instance
            std::vector<usbs_handle *> hs(act.size());
            std::vector<usbs::PackState> sts(act.size());
            const double now0 = sv->now();
            for (size_t q = 0; q < act.size(); ++q) {
                hs[q] = act[q].h;
                sts[q] = act[q].st;
                const double lim = sv->cfg.params.time_limit;
                if (lim > 0.0 && now0 - act[q].t_phase > lim) sts[q].stop = 1;
            }
            std::string err;
            const int rc = usbs_pack::launch(R, hs.data(), sts.data(), (int)act.size(), iters, &err);
            for (size_t q = 0; q < act.size(); ++q) {
                act[q].st = sts[q];
                if (rc < 0) act[q].st.done = usbs::PACK_FAILED;
            }
            if (rc < 0) {
                std::lock_guard<std::mutex> lk(sv->mu);
                sv->err = err;
            }
            // retire finished solves; warm restarts of grown instances stay in the table
            std::vector<Active> keep;
            for (Active &a : act) {
                if (a.st.done == usbs::PACK_RUNNING) {
                    keep.push_back(a);
                    continue;
                }
                const double secs = sv->now() - a.t_phase;
                Request *rq = a.rq;
                if (!a.grown) {
                    rq->status_base = rc < 0 ? rc : usbs_pack::finish(a.h, a.st, &rq->res_base, secs);
                    rq->t_base_done = sv->now();
                    if (rq->status_base >= 0 && rq->has_grown) {
                        usbs_problem pg = rq->grown.view();
                        const int st2 = usbs_pack::warm_prepare(a.h, &pg, false);
                        if (st2 == USBS_OK) {
                            a.grown = true;
                            a.t_phase = sv->now();
                            a.st = usbs_pack::begin(a.h, usbs::PACK_INIT_WARM);
                            keep.push_back(a);
                            continue;
                        }
                        rq->status_grown = st2;
                    }
                } else {
                    rq->status_grown = rc < 0 ? rc : usbs_pack::finish(a.h, a.st, &rq->res_grown, secs);
                }
                finish_request(sv, a);
            }
            act.swap(keep);
            sv->cv_work.notify_all();
        }
    }
    if (side_stream) (void)hipStreamDestroy(side_stream);
    if (launch_stream) (void)hipStreamDestroy(launch_stream);
}
}  // namespace

extern "C" {

int usbs_server_create(const usbs_server_config *cfg, usbs_server **out) {
    if (!out || !cfg) return USBS_E_INVALID;
    *out = nullptr;
    if (cfg->mode != USBS_SERVE_STREAMS && cfg->mode != USBS_SERVE_PACKED) return USBS_E_INVALID;
    if (cfg->large_slots > 16) return USBS_E_INVALID;
    if (cfg->slots < 1 || cfg->slots > (cfg->mode == USBS_SERVE_PACKED ? 1024 : 64)) return USBS_E_INVALID;
    auto *sv = new usbs_server();
    sv->cfg = *cfg;
    sv->t0 = std::chrono::steady_clock::now();
    if (hipGetDevice(&sv->dev) != hipSuccess) {
        delete sv;
        return USBS_E_DEVICE;
    }
    sv->budget = cfg->hbm_budget_bytes;
    if (sv->budget <= 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
            delete sv;
            return USBS_E_DEVICE;
        }
        sv->budget = (int64_t)(0.9 * (double)fr);
    }
    sv->packed = cfg->mode == USBS_SERVE_PACKED;
    sv->packed_max_n = cfg->packed_max_n > 0 ? cfg->packed_max_n : 20000;
    if (sv->packed) {
        sv->workers.emplace_back(packer, sv);
        const int large = cfg->large_slots < 0 ? 2 : cfg->large_slots;
        for (int q = 0; q < large; ++q) sv->workers.emplace_back(worker, sv, q);
    } else {
        for (int q = 0; q < cfg->slots; ++q) sv->workers.emplace_back(worker, sv, q);
    }
    *out = sv;
    return USBS_OK;
}

int usbs_server_submit(usbs_server *sv, const usbs_problem *prob, const usbs_problem *grown, int64_t *request_id) {
    if (!sv || !prob || !request_id) return USBS_E_INVALID;
    auto rq = std::make_unique<Request>();
    const int r = sv->cfg.params.r;
    rq->base.copy_from(prob, r);
    int64_t fp = usbs_footprint_bytes(prob, &sv->cfg.params);
    if (grown) {
        if (grown->n < prob->n || grown->m < prob->m) return USBS_E_INVALID;
        rq->grown.copy_from(grown, r);
        rq->has_grown = true;
        fp = std::max(fp, usbs_footprint_bytes(grown, &sv->cfg.params));
    }
    if (fp <= 0) return USBS_E_INVALID;
    std::lock_guard<std::mutex> lk(sv->mu);
    if (fp > sv->budget) {
        sv->err = "request footprint exceeds the server's HBM budget";
        return USBS_E_NOMEM;
    }
    rq->footprint = fp;
    rq->nmax = grown ? std::max(prob->n, grown->n) : prob->n;
    if (sv->packed && rq->nmax > sv->packed_max_n && sv->cfg.large_slots == 0) {
        sv->err = "request above packed_max_n and no per-instance worker (large_slots = 0)";
        return USBS_E_INVALID;
    }
    rq->id = sv->next_id++;
    rq->t_submit = sv->now();
    *request_id = rq->id;
    sv->queue.push_back(rq.get());
    sv->reqs[rq->id] = std::move(rq);
    sv->cv_work.notify_all();
    return USBS_OK;
}

int usbs_server_wait(usbs_server *sv, int64_t request_id, usbs_served_result *out) {
    if (!sv || !out) return USBS_E_INVALID;
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(request_id);
    if (it == sv->reqs.end()) return USBS_E_STATE;
    Request *rq = it->second.get();
    sv->cv_done.wait(lk, [&] { return rq->done; });
    std::memset(out, 0, sizeof(*out));
    out->base = rq->res_base;
    out->grown = rq->res_grown;
    out->status_base = rq->status_base;
    out->status_grown = rq->status_grown;
    out->has_grown = rq->has_grown ? 1 : 0;
    out->slot = rq->slot;
    out->footprint_bytes = rq->footprint;
    out->t_submit = rq->t_submit;
    out->t_admit = rq->t_admit;
    out->t_base_done = rq->t_base_done;
    out->t_done = rq->t_done;
    if (!rq->err.empty()) sv->err = rq->err;
    const int st = (rq->status_base < 0) ? rq->status_base : ((rq->status_grown < 0) ? rq->status_grown : USBS_OK);
    sv->reqs.erase(it);
    return st;
}

int usbs_server_get_stats(usbs_server *sv, usbs_server_stats *out) {
    if (!sv || !out) return USBS_E_INVALID;
    std::lock_guard<std::mutex> lk(sv->mu);
    out->queued = (int64_t)sv->queue.size();
    out->running = sv->running;
    out->peak_running = sv->peak_running;
    out->completed = sv->completed;
    out->budget_bytes = sv->budget;
    out->used_bytes = sv->used;
    out->peak_used_bytes = sv->peak_used;
    out->seconds = sv->now();
    return USBS_OK;
}

const char *usbs_server_last_error(const usbs_server *sv) { return sv ? sv->err.c_str() : "NULL server"; }

void usbs_server_free(usbs_server *sv) {
    if (!sv) return;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
    }
    sv->cv_work.notify_all();
    for (auto &t : sv->workers) t.join();
    delete sv;
}

}  // extern "C"
