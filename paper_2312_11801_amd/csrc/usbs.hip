// Host side of the USBS library: problem validation and scaling (App. E),
// device memory, the block Lanczos eigen-solver and the iteration of Alg. 1,
// all issued as kernels on one HIP stream.  Implements include/usbs.h.
#include "../../include/usbs.h"
#include "kernels.h"
#include "steps.h"
#include "packed.h"
#include "packed_host.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <stdexcept>
#include <string>
#include <utility>
#include <vector>

using namespace usbs;

namespace usbs_noalloc {
const char *last_error();   // noalloc.hip
}

namespace {

struct DevError : std::runtime_error {
    int code;
    DevError(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define HIPCHK(x)                                                                                      \
    do {                                                                                               \
        hipError_t e_ = (x);                                                                           \
        if (e_ != hipSuccess)                                                                          \
            throw DevError(e_ == hipErrorOutOfMemory ? USBS_E_NOMEM : USBS_E_DEVICE,                   \
                           std::string(#x) + ": " + hipGetErrorString(e_));                            \
    } while (0)

// Device memory is stream-ordered (hipMallocAsync / hipFreeAsync on the handle's stream):
// creating or releasing one handle never waits for work that other handles run on
// other streams (a plain hipFree synchronises the whole device).
template <typename T>
T *dalloc(size_t count, std::vector<void *> &owned, hipStream_t s) {
    void *p = nullptr;
    if (count == 0) count = 1;
    HIPCHK(hipMallocAsync(&p, count * sizeof(T), s));
    owned.push_back(p);
    return (T *)p;
}

// host copy of a problem (kept for warm starts)
struct HostProblem {
    int n = 0, m = 0;
    std::vector<int64_t> rowptr;
    std::vector<int32_t> col;
    std::vector<double> val;
    std::vector<int32_t> a_row, a_i, a_j;
    std::vector<double> a_v, b;
    std::vector<uint8_t> ineq;
    double trace = 0.0;
    std::vector<float> psi;   // n * r (empty without sketch)
};

}  // namespace

struct usbs_handle {
    std::string err;
    int dev = 0;
    hipStream_t stream = nullptr;
    usbs_params prm{};
    HostProblem hp;
    std::vector<void *> owned;   // device allocations of the current problem

    int n = 0, m = 0, nnz = 0, k = 0, kc = 0, kp = 0, r = 0, prec = 0, steps = 8, ldb = 80;
    bool sketch = false, has_offc = false, has_ineq = false;
    double sigma = 1.0, trace = 1.0, val_scale = 1.0, bnorm = 0.0;

    // operator (off-diagonal CSR, diagonal split out)
    int *rowptr = nullptr, *col = nullptr;
    void *val_cur = nullptr, *val_c = nullptr;   // compute precision: shifted / base
    double *cbase = nullptr, *cdiag = nullptr, *dshift = nullptr;
    int *dptr = nullptr, *dk = nullptr;
    double *dv = nullptr;
    int n_offt = 0;
    int *off_slot = nullptr, *off_ptr = nullptr, *off_k = nullptr;
    double *off_hv = nullptr;
    int *kptr = nullptr, *ti = nullptr, *tj = nullptr;
    double *tv = nullptr, *b = nullptr, *ineq = nullptr;
    float *psi = nullptr;

    // iteration state
    double *y = nullptr, *yc = nullptr, *nu = nullptr, *dnu = nullptr, *zbar = nullptr, *AX = nullptr,
           *evec = nullptr, *AXhat = nullptr;
    double *V = nullptr, *Vn = nullptr, *CV = nullptr, *Uritz = nullptr, *P = nullptr;
    // decoupled rows (exact eigenpairs (d_i, e_i)); Ucpl = Ritz vectors of the coupled
    // rows (the Lanczos state; aliases Uritz when there are no decoupled rows)
    int n_iso = 0;
    int *iso_idx = nullptr, *plan = nullptr;
    double *Ucpl = nullptr;
    // Lanczos work
    double *Bm = nullptr, *W = nullptr, *Wt = nullptr, *W2 = nullptr, *Ubuf = nullptr;
    double *Tm = nullptr, *theta = nullptr, *Ysm = nullptr, *TUU = nullptr, *RtR = nullptr, *Zc = nullptr,
           *Hred = nullptr, *Rinv = nullptr, *res = nullptr, *Hd = nullptr;
    double *Hg = nullptr, *coef = nullptr, *Rsv = nullptr;   // block Gram-Schmidt (Pythagorean) work
    double *Tscr = nullptr;                                   // projections of a fresh block (16 x 8, unused)
    int *skip2 = nullptr;                                     // the block step's second pass is left out
    int *dead = nullptr, *flag = nullptr;
    // QP / model
    double *raw = nullptr, *qp = nullptr, *ipm = nullptr, *VCV = nullptr, *Gy = nullptr, *Kc = nullptr,
           *Qp = nullptr, *Hsk = nullptr, *VtPsi = nullptr, *sc = nullptr, *small = nullptr, *Zp = nullptr,
           *hz = nullptr, *Rz = nullptr, *Qp8 = nullptr;
    int *zdead = nullptr;
    RedScratch rs{};
    // side stream (default priority) for V^T Psi, which runs beside the one-workgroup master-QP
    // solve; its own reduction scratch
    hipStream_t side = nullptr;
    hipEvent_t ev_side0 = nullptr, ev_side1 = nullptr, ev_side2 = nullptr;
    RedScratch rs_side{};

    Tuning tune;   // launch shapes (autotuner)

    int64_t matvecs = 0;
    uint64_t pack_ticks[kPackPhases] = {};   // device wall-clock ticks per phase of packed launches
    int iters = 0;
    int lz_unconverged = 0;   // in-iteration eigen-solves that hit the restart limit
    int null_run = 0;         // consecutive null steps
    int recoveries = 0;       // stall re-evaluations of f at the centre
    bool last_conv = false;
    bool conv_pending = false;   // last_conv is still on its way into conv_host
    int *conv_host = nullptr;    // pinned
    bool ready = false;
    // value of iters after which AX, Vn (= V_t) and the QP solution in ipm describe
    // X_{t+1} of that iteration; -1 before the first iteration of the current problem
    int primal_at = -1;

    // live timing of one kernel category with HIP events (bench / roofline)
    int prof_cat = -1;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    double prof_ms = 0.0;
    int64_t prof_count = 0;
};

void nn_update_dev_beta(usbs_handle *h, const double *A, int lda, int ca, const double *H, int ldh, int cc, double *C,
                        int ldc);

namespace {

// RAII: records a start/stop event pair around the launches of the profiled category
struct ProfScope {
    usbs_handle *h;
    int idx = -1;
    ProfScope(usbs_handle *hh, int cat) : h(hh) {
        if (h->prof_cat != cat) return;
        if (h->ev_used + 2 > h->ev_pool.size()) return;
        idx = (int)h->ev_used;
        h->ev_used += 2;
        (void)hipEventRecord(h->ev_pool[idx], h->stream);
    }
    ~ProfScope() {
        if (idx >= 0) (void)hipEventRecord(h->ev_pool[idx + 1], h->stream);
    }
};

// event pair for a launch that records its own start / end (hipExtLaunchKernelGGL)
struct ProfPair {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ProfPair(usbs_handle *h, int cat) {
        if (h->prof_cat != cat) return;
        if (h->ev_used + 2 > h->ev_pool.size()) return;
        e0 = h->ev_pool[h->ev_used];
        e1 = h->ev_pool[h->ev_used + 1];
        h->ev_used += 2;
    }
};

void prof_flush(usbs_handle *h) {
    if (h->ev_used == 0) return;
    (void)hipEventSynchronize(h->ev_pool[h->ev_used - 1]);
    for (size_t q = 0; q + 1 < h->ev_used; q += 2) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, h->ev_pool[q], h->ev_pool[q + 1]) == hipSuccess) {
            h->prof_ms += ms;
            h->prof_count++;
        }
    }
    h->ev_used = 0;
}

void set_err(usbs_handle *h, const std::string &m) {
    if (h) h->err = m;
}

// ---------------------------------------------------------------------------
// validation and upload
// ---------------------------------------------------------------------------
HostProblem copy_problem(const usbs_problem *p, int r) {
    if (!p) throw DevError(USBS_E_INVALID, "problem is NULL");
    if (p->n < 2 || p->n > (int64_t)1 << 30) throw DevError(USBS_E_INVALID, "n out of range");
    if (p->m < 1 || p->m > (int64_t)1 << 30) throw DevError(USBS_E_INVALID, "m out of range");
    if (!p->rowptr || !p->col || !p->val || !p->b || !p->is_ineq)
        throw DevError(USBS_E_INVALID, "NULL array in problem");
    if (p->n_triplets < 1 || !p->a_row || !p->a_i || !p->a_j || !p->a_v)
        throw DevError(USBS_E_INVALID, "constraint triplets missing");
    if (!(p->trace > 0.0) || !std::isfinite(p->trace)) throw DevError(USBS_E_INVALID, "trace must be > 0");
    HostProblem hp;
    hp.n = (int)p->n;
    hp.m = (int)p->m;
    const int64_t nnz = p->rowptr[p->n];
    if (p->rowptr[0] != 0 || nnz < 0 || nnz >= ((int64_t)1 << 31)) throw DevError(USBS_E_INVALID, "bad rowptr");
    hp.rowptr.assign(p->rowptr, p->rowptr + p->n + 1);
    for (int64_t i = 0; i < p->n; ++i)
        if (hp.rowptr[i + 1] < hp.rowptr[i]) throw DevError(USBS_E_INVALID, "rowptr not monotone");
    hp.col.assign(p->col, p->col + nnz);
    hp.val.assign(p->val, p->val + nnz);
    for (int64_t e = 0; e < nnz; ++e) {
        if (hp.col[e] < 0 || hp.col[e] >= p->n) throw DevError(USBS_E_INVALID, "column index out of range");
        if (!std::isfinite(hp.val[e])) throw DevError(USBS_E_NUMERIC, "non-finite value in C");
    }
    const int64_t nt = p->n_triplets;
    hp.a_row.assign(p->a_row, p->a_row + nt);
    hp.a_i.assign(p->a_i, p->a_i + nt);
    hp.a_j.assign(p->a_j, p->a_j + nt);
    hp.a_v.assign(p->a_v, p->a_v + nt);
    for (int64_t t = 0; t < nt; ++t) {
        if (hp.a_row[t] < 0 || hp.a_row[t] >= p->m || hp.a_i[t] < 0 || hp.a_j[t] >= p->n ||
            hp.a_i[t] > hp.a_j[t])
            throw DevError(USBS_E_INVALID, "constraint triplet out of range (need 0 <= i <= j < n)");
        if (!std::isfinite(hp.a_v[t])) throw DevError(USBS_E_NUMERIC, "non-finite constraint coefficient");
    }
    hp.b.assign(p->b, p->b + p->m);
    hp.ineq.assign(p->is_ineq, p->is_ineq + p->m);
    for (int k = 0; k < hp.m; ++k)
        if (!std::isfinite(hp.b[k])) throw DevError(USBS_E_NUMERIC, "non-finite b");
    hp.trace = p->trace;
    if (p->psi) {
        hp.psi.assign(p->psi, p->psi + (size_t)p->n * r);
        for (float v : hp.psi)
            if (!std::isfinite(v)) throw DevError(USBS_E_NUMERIC, "non-finite test matrix");
    }
    // C symmetric (pattern and values)
    {
        std::vector<std::pair<int64_t, double>> tr;
        tr.reserve(nnz);
        std::vector<std::pair<int64_t, double>> fw;
        fw.reserve(nnz);
        for (int i = 0; i < hp.n; ++i)
            for (int64_t e = hp.rowptr[i]; e < hp.rowptr[i + 1]; ++e) {
                const int j = hp.col[e];
                fw.push_back({(int64_t)i * hp.n + j, hp.val[e]});
                tr.push_back({(int64_t)j * hp.n + i, hp.val[e]});
            }
        std::sort(fw.begin(), fw.end());
        std::sort(tr.begin(), tr.end());
        for (size_t e = 0; e < fw.size(); ++e) {
            if (e > 0 && fw[e].first == fw[e - 1].first) throw DevError(USBS_E_INVALID, "duplicate entry in C");
            if (fw[e].first != tr[e].first || std::fabs(fw[e].second - tr[e].second) >
                                                  1e-12 * (1.0 + std::fabs(fw[e].second)))
                throw DevError(USBS_E_INVALID, "C is not symmetric");
        }
    }
    return hp;
}

void free_problem(usbs_handle *h) {
    for (void *p : h->owned) (void)hipFreeAsync(p, h->stream);
    (void)hipStreamSynchronize(h->stream);
    h->owned.clear();
}

void upload(usbs_handle *h) {
    const HostProblem &hp = h->hp;
    const int n = hp.n, m = hp.m;
    h->n = n;
    h->m = m;
    std::vector<void *> &o = h->owned;
    // scaling (App. E, eq. std_scaling)
    double fro2 = 0.0;
    for (double v : hp.val) fro2 += v * v;
    h->sigma = fro2 > 0.0 ? std::sqrt(fro2) : 1.0;
    h->trace = hp.trace;
    double bn2 = 0.0;
    for (double v : hp.b) bn2 += (v / hp.trace) * (v / hp.trace);
    h->bnorm = std::sqrt(bn2);
    h->has_ineq = false;
    for (uint8_t v : hp.ineq) h->has_ineq |= (v != 0);

    // off-diagonal pattern: C's off-diagonal entries plus the pairs that constraints touch
    std::vector<double> cdiag(n, 0.0);
    std::vector<std::vector<std::pair<int, double>>> rows(n);
    for (int i = 0; i < n; ++i)
        for (int64_t e = hp.rowptr[i]; e < hp.rowptr[i + 1]; ++e) {
            const int j = hp.col[e];
            if (j == i) cdiag[i] += hp.val[e] / h->sigma;
            else rows[i].push_back({j, hp.val[e] / h->sigma});
        }
    // constraint triplets: diagonal ones per vertex, off-diagonal ones per slot
    std::vector<std::vector<std::pair<int, double>>> dlist(n);
    struct OffT { int i, j, k; double hv; };
    std::vector<OffT> offt;
    for (size_t t = 0; t < hp.a_row.size(); ++t) {
        const int i = hp.a_i[t], j = hp.a_j[t], k = hp.a_row[t];
        if (i == j) dlist[i].push_back({k, hp.a_v[t]});
        else offt.push_back({i, j, k, 0.5 * hp.a_v[t]});
    }
    // decoupled rows: no nonzero off-diagonal of C and no constraint touching an
    // off-diagonal pair, so C - A^*(y) is diagonal on them for every y
    std::vector<char> coupled(n, 0);
    for (int i = 0; i < n; ++i)
        for (auto &pr : rows[i]) coupled[i] |= (pr.second != 0.0);
    for (auto &ot : offt) coupled[ot.i] = coupled[ot.j] = 1;
    std::vector<int> iso;
    for (int i = 0; i < n; ++i)
        if (!coupled[i]) iso.push_back(i);
    h->n_iso = (int)iso.size();
    if (h->n_iso < n && n - h->n_iso < 2 * (16 + 8))
        throw DevError(USBS_E_INVALID, "too few coupled rows for the block Lanczos basis (need 0 or >= 48)");
    for (auto &ot : offt) {
        bool f1 = false, f2 = false;
        for (auto &pr : rows[ot.i]) f1 |= (pr.first == ot.j);
        for (auto &pr : rows[ot.j]) f2 |= (pr.first == ot.i);
        if (!f1) rows[ot.i].push_back({ot.j, 0.0});
        if (!f2) rows[ot.j].push_back({ot.i, 0.0});
    }
    for (int i = 0; i < n; ++i) std::sort(rows[i].begin(), rows[i].end());
    std::vector<int> rp(n + 1, 0);
    for (int i = 0; i < n; ++i) rp[i + 1] = rp[i] + (int)rows[i].size();
    const int nnz = rp[n];
    h->nnz = nnz;
    std::vector<int> colv(std::max(nnz, 1));
    std::vector<double> cb(std::max(nnz, 1));
    for (int i = 0; i < n; ++i)
        for (size_t q = 0; q < rows[i].size(); ++q) {
            colv[rp[i] + q] = rows[i][q].first;
            cb[rp[i] + q] = rows[i][q].second;
        }
    auto slot_of = [&](int i, int j) -> int {
        auto it = std::lower_bound(colv.begin() + rp[i], colv.begin() + rp[i + 1], j);
        return (int)(it - colv.begin());
    };
    // constrained off-diagonal slots: both CSR slots of every off-diagonal triplet, grouped
    // by slot (a pair may appear in several rows), so that each slot's value
    // c_ij - sum_k (v_k / 2) y_k is formed by one thread in a fixed order
    std::vector<int> osl, ok, optr;
    std::vector<double> ohv;
    {
        struct SlotEntry { int slot, k; double hv; };
        std::vector<SlotEntry> ent;
        ent.reserve(2 * offt.size());
        for (auto &ot : offt) {
            ent.push_back({slot_of(ot.i, ot.j), ot.k, ot.hv});
            ent.push_back({slot_of(ot.j, ot.i), ot.k, ot.hv});
        }
        std::stable_sort(ent.begin(), ent.end(), [](const SlotEntry &a, const SlotEntry &b) { return a.slot < b.slot; });
        for (size_t t = 0; t < ent.size(); ++t) {
            if (t == 0 || ent[t].slot != ent[t - 1].slot) {
                osl.push_back(ent[t].slot);
                optr.push_back((int)t);
            }
            ok.push_back(ent[t].k);
            ohv.push_back(ent[t].hv);
        }
        optr.push_back((int)ent.size());
    }
    h->n_offt = (int)osl.size();   // constrained slots
    h->has_offc = h->n_offt > 0;
    std::vector<int> dp(n + 1, 0), dkv;
    std::vector<double> dvv;
    for (int i = 0; i < n; ++i) {
        for (auto &pr : dlist[i]) {
            dkv.push_back(pr.first);
            dvv.push_back(pr.second);
        }
        dp[i + 1] = (int)dkv.size();
    }
    // constraint rows as CSR over triplets
    std::vector<int> kp(m + 1, 0);
    for (int v : hp.a_row) kp[v + 1]++;
    for (int k = 0; k < m; ++k) kp[k + 1] += kp[k];
    std::vector<int> tiv(hp.a_row.size()), tjv(hp.a_row.size());
    std::vector<double> tvv(hp.a_row.size());
    {
        std::vector<int> pos(kp.begin(), kp.end() - 1);
        for (size_t t = 0; t < hp.a_row.size(); ++t) {
            const int q = pos[hp.a_row[t]]++;
            tiv[q] = hp.a_i[t];
            tjv[q] = hp.a_j[t];
            tvv[q] = hp.a_v[t];
        }
    }
    // BF16 values carry a common factor so that equal magnitudes stay exact
    double mx = 0.0;
    for (int e = 0; e < nnz; ++e) mx = std::max(mx, std::fabs(cb[e]));
    h->val_scale = (h->prec == USBS_PREC_BF16 && mx > 0.0) ? mx : 1.0;

    hipStream_t s = h->stream;
    h->rowptr = dalloc<int>(n + 1, o, h->stream);
    h->col = dalloc<int>(nnz, o, h->stream);
    h->cbase = dalloc<double>(nnz, o, h->stream);
    const size_t vsz = h->prec == 0 ? 8 : (h->prec == 1 ? 4 : 2);
    h->val_cur = dalloc<char>(std::max(nnz, 1) * vsz, o, h->stream);
    h->val_c = h->has_offc ? (void *)dalloc<char>(std::max(nnz, 1) * vsz, o, h->stream) : h->val_cur;
    h->cdiag = dalloc<double>(n, o, h->stream);
    h->dshift = dalloc<double>(n, o, h->stream);
    h->dptr = dalloc<int>(n + 1, o, h->stream);
    h->dk = dalloc<int>(dkv.size(), o, h->stream);
    h->dv = dalloc<double>(dvv.size(), o, h->stream);
    h->off_slot = dalloc<int>(osl.size(), o, h->stream);
    h->off_ptr = dalloc<int>(optr.size(), o, h->stream);
    h->off_k = dalloc<int>(ok.size(), o, h->stream);
    h->off_hv = dalloc<double>(ohv.size(), o, h->stream);
    h->kptr = dalloc<int>(m + 1, o, h->stream);
    h->ti = dalloc<int>(tiv.size(), o, h->stream);
    h->tj = dalloc<int>(tjv.size(), o, h->stream);
    h->tv = dalloc<double>(tvv.size(), o, h->stream);
    h->b = dalloc<double>(m, o, h->stream);
    h->ineq = dalloc<double>(m, o, h->stream);
    HIPCHK(hipMemcpyAsync(h->rowptr, rp.data(), (n + 1) * sizeof(int), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(h->col, colv.data(), nnz * sizeof(int), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(h->cbase, cb.data(), nnz * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(h->cdiag, cdiag.data(), n * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(h->dptr, dp.data(), (n + 1) * sizeof(int), hipMemcpyHostToDevice, s));
    if (!dkv.empty()) {
        HIPCHK(hipMemcpyAsync(h->dk, dkv.data(), dkv.size() * sizeof(int), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(h->dv, dvv.data(), dvv.size() * sizeof(double), hipMemcpyHostToDevice, s));
    }
    if (!osl.empty()) {
        HIPCHK(hipMemcpyAsync(h->off_slot, osl.data(), osl.size() * sizeof(int), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(h->off_ptr, optr.data(), optr.size() * sizeof(int), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(h->off_k, ok.data(), ok.size() * sizeof(int), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(h->off_hv, ohv.data(), ohv.size() * sizeof(double), hipMemcpyHostToDevice, s));
    }
    HIPCHK(hipMemcpyAsync(h->kptr, kp.data(), (m + 1) * sizeof(int), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(h->ti, tiv.data(), tiv.size() * sizeof(int), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(h->tj, tjv.data(), tjv.size() * sizeof(int), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(h->tv, tvv.data(), tvv.size() * sizeof(double), hipMemcpyHostToDevice, s));
    std::vector<double> bs(m), inq(m);
    for (int k = 0; k < m; ++k) {
        bs[k] = hp.b[k] / hp.trace;
        inq[k] = hp.ineq[k] ? 1.0 : 0.0;
    }
    HIPCHK(hipMemcpyAsync(h->b, bs.data(), m * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(h->ineq, inq.data(), m * sizeof(double), hipMemcpyHostToDevice, s));
    h->sketch = h->r > 0;
    if (h->sketch) {
        h->psi = dalloc<float>((size_t)n * h->r, o, h->stream);
        if (!hp.psi.empty())
            HIPCHK(hipMemcpyAsync(h->psi, hp.psi.data(), (size_t)n * h->r * sizeof(float), hipMemcpyHostToDevice,
                                  s));
        else
            psi_from_seed(s, n, h->r, h->prm.psi_seed, h->psi);   // Sec. 4 test matrix, generated here
    }
    convert_values(s, h->prec, nnz, h->cbase, 1.0 / h->val_scale, h->val_cur);
    if (h->has_offc) convert_values(s, h->prec, nnz, h->cbase, 1.0 / h->val_scale, h->val_c);

    // state and work arrays
    const int ldb = h->ldb;
    h->y = dalloc<double>(m, o, h->stream);
    h->yc = dalloc<double>(m, o, h->stream);
    h->nu = dalloc<double>(m, o, h->stream);
    h->dnu = dalloc<double>(m, o, h->stream);
    h->zbar = dalloc<double>(m, o, h->stream);
    h->AX = dalloc<double>(m, o, h->stream);
    h->AXhat = dalloc<double>(m, o, h->stream);
    h->evec = dalloc<double>(m, o, h->stream);
    h->V = dalloc<double>((size_t)n * 16, o, h->stream);
    h->Vn = dalloc<double>((size_t)n * 16, o, h->stream);
    h->CV = dalloc<double>((size_t)n * 16, o, h->stream);
    h->Uritz = dalloc<double>((size_t)n * 16, o, h->stream);
    h->plan = dalloc<int>(16, o, h->stream);
    if (h->n_iso > 0) {
        h->iso_idx = dalloc<int>(h->n_iso, o, h->stream);
        HIPCHK(hipMemcpyAsync(h->iso_idx, iso.data(), h->n_iso * sizeof(int), hipMemcpyHostToDevice, s));
        h->Ucpl = dalloc<double>((size_t)n * 16, o, h->stream);
        HIPCHK(hipMemsetAsync(h->Ucpl, 0, (size_t)n * 16 * sizeof(double), s));
    } else {
        h->iso_idx = nullptr;
        h->Ucpl = h->Uritz;
    }
    h->P = dalloc<double>((size_t)n * std::max(h->r, 1), o, h->stream);
    h->Bm = dalloc<double>((size_t)n * ldb, o, h->stream);
    h->W = dalloc<double>((size_t)n * 8, o, h->stream);
    h->Wt = dalloc<double>((size_t)n * 8, o, h->stream);
    h->W2 = dalloc<double>((size_t)n * 32, o, h->stream);
    h->Ubuf = dalloc<double>((size_t)n * 16, o, h->stream);
    h->Zp = dalloc<double>((size_t)n * 16, o, h->stream);
    h->Tm = dalloc<double>((size_t)ldb * ldb, o, h->stream);
    h->theta = dalloc<double>(ldb, o, h->stream);
    h->Ysm = dalloc<double>((size_t)ldb * 16, o, h->stream);
    h->TUU = dalloc<double>(256, o, h->stream);
    h->RtR = dalloc<double>(256, o, h->stream);
    h->Zc = dalloc<double>(128, o, h->stream);
    h->Hred = dalloc<double>((size_t)ldb * 16, o, h->stream);
    h->Hg = dalloc<double>((size_t)(ldb + 8) * 8, o, h->stream);
    h->coef = dalloc<double>((size_t)(ldb + 8) * 8, o, h->stream);
    h->Rsv = dalloc<double>(64, o, h->stream);
    h->Tscr = dalloc<double>(16 * 8, o, h->stream);
    h->skip2 = dalloc<int>(1, o, h->stream);
    h->Rinv = dalloc<double>(256, o, h->stream);
    h->res = dalloc<double>(16, o, h->stream);
    h->Hd = dalloc<double>(256, o, h->stream);
    h->dead = dalloc<int>(ldb, o, h->stream);
    h->flag = dalloc<int>(24, o, h->stream);   // 16 start-block flags + 8 for a fresh block at column 16
    h->zdead = dalloc<int>(16, o, h->stream);
    const int d = kMaxSvec;
    h->raw = dalloc<double>(d * d + 4 * d, o, h->stream);
    h->qp = dalloc<double>(d * d + 2 * d + 2, o, h->stream);
    h->ipm = dalloc<double>(2 * kMaxK * kMaxK + 8, o, h->stream);
    h->VCV = dalloc<double>(256, o, h->stream);
    h->Gy = dalloc<double>(d * d + 4 * d, o, h->stream);
    h->Kc = dalloc<double>(256, o, h->stream);
    h->Qp = dalloc<double>(256, o, h->stream);
    h->Qp8 = dalloc<double>(16 * 8, o, h->stream);
    h->Hsk = dalloc<double>(16 * 32, o, h->stream);
    h->VtPsi = dalloc<double>(16 * 32, o, h->stream);
    h->hz = dalloc<double>(256, o, h->stream);
    h->Rz = dalloc<double>(256, o, h->stream);
    h->sc = dalloc<double>(SC_COUNT, o, h->stream);
    h->small = dalloc<double>(4096, o, h->stream);
    h->rs.max_blocks = kRedMaxBlocks;
    h->rs.max_elems = kMaxSvec * (kMaxSvec + 1) / 2 + 4 * kMaxSvec;
    if (h->rs.max_elems < kMaxBasis * 16) h->rs.max_elems = kMaxBasis * 16;
    h->rs.partials = dalloc<double>((size_t)h->rs.max_blocks * h->rs.max_elems, o, h->stream);
    h->rs.counter = dalloc<unsigned>(4, o, h->stream);
    h->rs_side.max_blocks = kRedMaxBlocks;
    h->rs_side.max_elems = h->rs.max_elems;
    h->rs_side.partials = dalloc<double>((size_t)h->rs_side.max_blocks * h->rs_side.max_elems, o, h->stream);
    HIPCHK(hipMemsetAsync(h->rs.counter, 0, 4 * sizeof(unsigned), s));
    HIPCHK(hipMemsetAsync(h->V, 0, (size_t)n * 16 * sizeof(double), s));
    HIPCHK(hipMemsetAsync(h->Vn, 0, (size_t)n * 16 * sizeof(double), s));
    HIPCHK(hipMemsetAsync(h->CV, 0, (size_t)n * 16 * sizeof(double), s));
    HIPCHK(hipMemsetAsync(h->P, 0, (size_t)n * std::max(h->r, 1) * sizeof(double), s));
    HIPCHK(hipMemsetAsync(h->nu, 0, m * sizeof(double), s));
    HIPCHK(hipMemsetAsync(h->Bm, 0, (size_t)n * ldb * sizeof(double), s));
}

// ---------------------------------------------------------------------------
// operator pieces
// ---------------------------------------------------------------------------
void shift_operator(usbs_handle *h, const double *y) {
    diag_shift(h->stream, h->n, h->dptr, h->dk, h->dv, h->cdiag, y, h->dshift);
    if (h->has_offc)
        offdiag_refresh(h->stream, h->prec, h->n_offt, h->off_slot, h->off_ptr, h->off_k, h->off_hv, h->cbase, y,
                        1.0 / h->val_scale, h->val_cur);
    // scale of the Lanczos tolerances and of the Cholesky-QR deflation floor
    op_bound(h->stream, h->rs, h->prec, h->n, h->rowptr, h->val_cur, h->val_scale, h->dshift, h->sc + SC_SCALE);
}

void apply_op(usbs_handle *h, const double *X, int ldx, double *Y, int ldy, int nb) {
    ProfScope ps(h, USBS_PROF_SPMM);
    if (h->ev_used + 2 > h->ev_pool.size()) prof_flush(h);
    spmm(h->stream, h->prec, h->n, h->rowptr, h->col, h->val_cur, h->val_scale, h->dshift, X, ldx, Y, ldy, nb);
    h->matvecs += nb;
}

void apply_C(usbs_handle *h, const double *X, int ldx, double *Y, int ldy, int nb) {
    spmm(h->stream, h->prec, h->n, h->rowptr, h->col, h->val_c, h->val_scale, h->cdiag, X, ldx, Y, ldy, nb);
}

// Cholesky-QR twice of the n x nc block src (ld lds) into dst (ld ldd); deflated
// columns are zero and flagged in flags[0..nc)
void cholqr2(usbs_handle *h, const double *src, int lds, int nc, double *tmp, int ldt, double *dst, int ldd,
             int *flags) {
    hipStream_t s = h->stream;
    tn_reduce(s, h->rs, h->n, src, lds, nc, src, lds, nc, h->Rinv, nc, 1.0, 0.0, 1, flags, h->sc + SC_SCALE);
    nn_update(s, h->n, src, lds, nc, h->Rinv, nc, nc, tmp, ldt, 1.0, 0.0);
    tn_reduce(s, h->rs, h->n, tmp, ldt, nc, tmp, ldt, nc, h->Rinv, nc, 1.0, 0.0, 1, flags, nullptr);
    nn_update(s, h->n, tmp, ldt, nc, h->Rinv, nc, nc, dst, ldd, 1.0, 0.0);
}

// Orthonormalise the fresh block W (n x 8, ld 8; zero beyond its used columns) against the
// orthonormal columns Q (n x nq, ld ldq) by two passes of block Gram-Schmidt with Pythagorean
// inner products, as in the Krylov block steps, and write its first cc columns to dst (ld ldd,
// disjoint from Q's columns).  Three sweeps over [Q W]: the reduction [Q W]^T W, the first
// update fused with the second pass's reduction, the second update.  Deflated columns are
// zero and flagged in flags[0..8) (zero padding columns always are); the projections go to T
// (nq x 8, ld ldt).  Uses W, Wt, Hg, coef and Rsv.  With cc == 8 the pass-0 block goes
// straight to dst and the second update runs only when pass 0 lost too much (kPass2Skip).
void orth_fresh(usbs_handle *h, const double *Q, int ldq, int nq, double *dst, int ldd, int cc, int *flags,
                double *T, int ldt) {
    hipStream_t s = h->stream;
    const int n = h->n;
    const bool direct = cc == 8;
    double *mid = direct ? dst : h->Wt;
    const int ldm = direct ? ldd : 8;
    int g = reorth_partials(s, h->rs, n, Q, ldq, nq, h->W, 8, 8);
    finish_pip(s, h->rs, g, nq, h->Hg, 0, h->Rsv, T, ldt, h->coef, flags, h->sc + SC_SCALE,
               direct ? h->skip2 : nullptr);
    g = nn_update2_reorth(s, h->rs, n, Q, ldq, nq, h->W, 8, h->coef, 8, mid, ldm);
    finish_pip(s, h->rs, g, nq, h->Hg, 1, h->Rsv, T, ldt, h->coef, flags, nullptr);
    nn_update2(s, n, Q, ldq, nq, mid, ldm, 8, h->coef, 8, cc, dst, ldd, direct ? h->skip2 : nullptr);
}

// ---------------------------------------------------------------------------
// block Lanczos with Rayleigh-Ritz restarts (the eigen step behind f(y),
// Sec. 3 and App. E): start block of 16 vectors, block width 8, 'steps'
// blocks per cycle, full FP64 re-orthogonalisation (two classical
// Gram-Schmidt passes), Cholesky-QR2 for each new block.  On return
// Uritz (n x 16) holds the Ritz vectors, theta[0..16) the Ritz values.
// The iteration runs on the coupled rows only (start block masked, an invariant
// subspace of the operator); the exact eigenpairs of the decoupled rows are
// merged in at the end, and Ucpl keeps the coupled Ritz vectors for the next
// start.
// ---------------------------------------------------------------------------
// keep < 16: the first keep (>= 8) columns of the start block are orthonormal (coupled Ritz
// vectors of an earlier solve) and h->W holds 16 - keep fresh directions, zero-padded to 8
// columns; with orth_start they are orthonormalised against the kept ones into the block's
// last columns (three sweeps instead of a Cholesky-QR2 of all 16).
// defer_last: the last allowed cycle ends the solve whatever its residual test says, so its
// flag is copied into h->conv_host for the caller to read at its next synchronisation
// (h->conv_pending) instead of the host waiting for the device here.
// stag > 0: the solve also ends, once min_cyc cycles are done, when the top Ritz value moved by
// at most stag * |theta_1| over the last cycle (a clustered top eigenvalue whose Ritz value has
// settled long before any single Ritz vector meets a tight residual test).
int lanczos(usbs_handle *h, const double *start, int kc, double tol, double tol_rest, int maxr, bool orth_start,
            int min_cyc, int keep = 16, bool defer_last = false, double stag = 0.0) {
    hipStream_t s = h->stream;
    const int n = h->n, ldb = h->ldb, steps = h->steps;
    if (start != h->Ubuf) copy_cols(s, n, start, 16, 16, h->Ubuf, 16);
    if (h->n_iso > 0) {
        mask_rows(s, h->n_iso, h->iso_idx, h->Ubuf, 16, 16);
        if (keep < 16) mask_rows(s, h->n_iso, h->iso_idx, h->W, 8, 8);
        orth_start = true;
        if (h->n_iso == n) {   // a diagonal operator: every eigenpair is exact
            iso_merge(s, h->n_iso, h->iso_idx, h->dshift, 0, h->theta, h->res, h->plan);
            gather_ritz(s, n, h->Ucpl, h->plan, h->Uritz);
            h->last_conv = true;
            return 0;
        }
    }
    if (orth_start) {
        set_int(s, h->flag, 24, 0);
        if (keep >= 8 && keep < 16)
            orth_fresh(h, h->Ubuf, 16, keep, h->Ubuf + keep, 16, 16 - keep, h->flag + keep, h->Tscr, 8);
        else cholqr2(h, h->Ubuf, 16, 16, h->W2, 16, h->Ubuf, 16, h->flag);
    }
    int cyc = 0;
    double th_prev = 0.0, th_now = 0.0;
    for (cyc = 0; cyc <= maxr; ++cyc) {
        // explicit Rayleigh-Ritz on span(U) and residuals
        apply_op(h, h->Ubuf, 16, h->W2, 16, 16);
        tn_reduce(s, h->rs, n, h->Ubuf, 16, 16, h->W2, 16, 16, h->TUU, 16, 1.0, 0.0);
        // after a cycle, U holds Ritz vectors of the explicit projection, so U^T M U is
        // diagonal up to rounding; the 16 x 16 eigenproblem is needed for a new start
        // block and for tight tolerances only
        // (in the first cycle, columns deflated by the start orthonormalisation are flagged)
        if (cyc == 0 || tol < 1e-7)
            small_eig(s, 16, h->TUU, 16, h->theta, h->Ysm, 16, 16, (cyc == 0 && orth_start) ? h->flag : nullptr);
        else diag_theta(s, h->TUU, 16, h->theta, h->Ysm);
        // Ritz vectors B = U Y into the basis, residuals R = M U Y - B Theta over U, R^T R
        rr_update(s, h->rs, n, h->Ubuf, h->W2, h->Ysm, h->theta, h->Bm, ldb, h->Ubuf, h->RtR);
        lanczos_restart_prep(s, h->RtR, h->theta, kc, tol, tol_rest, h->res, h->flag, h->Zc, h->sc + SC_SCALE);
        if (cyc == maxr && defer_last) {
            if (!h->conv_host) HIPCHK(hipHostMalloc((void **)&h->conv_host, sizeof(int), hipHostMallocDefault));
            HIPCHK(hipMemcpyAsync(h->conv_host, h->flag, sizeof(int), hipMemcpyDeviceToHost, s));
            h->conv_pending = true;
            break;
        }
        int conv = 0;
        HIPCHK(hipMemcpyAsync(&conv, h->flag, sizeof(int), hipMemcpyDeviceToHost, s));
        if (stag > 0) HIPCHK(hipMemcpyAsync(&th_now, h->theta, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        h->last_conv = conv != 0;
        const bool flat = stag > 0 && cyc > 0 && std::fabs(th_now - th_prev) <= stag * std::fabs(th_now);
        if (stag > 0 && h->prm.verbose)
            std::fprintf(stderr, "  re-evaluation cycle %d theta_1 %.16e conv %d\n", cyc, th_now, conv);
        th_prev = th_now;
        if (((conv || flat) && cyc >= min_cyc) || cyc == maxr) break;
        // Krylov expansion from the dominant residual directions W = U Zc, orthonormalised
        // against the 16 Ritz vectors by the two Pythagorean Gram-Schmidt passes of the block
        // steps below (three sweeps over [B W]).  Their projections land in T[0:16, 16:24],
        // which block step 0 overwrites with the projections of M q_0.
        lanczos_reset_T(s, h->Tm, ldb, ldb, h->theta, h->dead);
        nn_update(s, n, h->Ubuf, 16, 16, h->Zc, 8, 8, h->W, 8, 1.0, 0.0);
        orth_fresh(h, h->Bm, ldb, 16, h->Bm + 16, ldb, 8, h->dead + 16, h->Tm + 16, ldb);
        // block steps: W = M q_j, then two passes of block Gram-Schmidt with Pythagorean
        // inner products against the whole basis (one reduction [Q W]^T W per pass)
        for (int j = 0; j < steps; ++j) {
            const int c0 = 16 + 8 * j, cols = c0 + 8;
            const bool last = j == steps - 1;
            apply_op(h, h->Bm + c0, ldb, h->W, 8, 8);
            if (h->ev_used + 4 > h->ev_pool.size()) prof_flush(h);
            // pass 0: [Q W]^T W, Cholesky of the Pythagorean Gram matrix
            int g;
            {
                ProfPair pp(h, USBS_PROF_REORTH);
                g = reorth_partials(s, h->rs, n, h->Bm, ldb, cols, h->W, 8, 8, pp.e0, pp.e1);
            }
            finish_pip(s, h->rs, g, cols, h->Hg, 0, h->Rsv, h->Tm + c0, ldb, h->coef, nullptr, h->sc + SC_SCALE,
                       last ? nullptr : h->skip2);
            // pass-0 update Wt = [Q W] coef fused with pass 1's reduction [Q Wt]^T Wt (the
            // basis rows are read once for both)
            {
                ProfPair pp(h, USBS_PROF_UPDATE);
                // the pass-0 block goes straight into its basis slot (the next block): when pass 0
                // lost little it stays as it is, otherwise pass 1 corrects it in place
                g = nn_update2_reorth(s, h->rs, n, h->Bm, ldb, cols, h->W, 8, h->coef, 8, last ? h->Wt : h->Bm + cols,
                                      last ? 8 : ldb, pp.e0, pp.e1);
            }
            finish_pip(s, h->rs, g, cols, h->Hg, 1, h->Rsv, h->Tm + c0, ldb, h->coef, !last ? h->dead + cols : nullptr,
                       nullptr);
            if (!last)
                nn_update2(s, n, h->Bm, ldb, cols, h->Bm + cols, ldb, 8, h->coef, 8, 8, h->Bm + cols, ldb, h->skip2);
        }
        {
            ProfScope ps(h, USBS_PROF_RITZ);
            small_eig(s, ldb, h->Tm, ldb, h->theta, h->Ysm, 16, 16, h->dead);
        }
        nn_update(s, n, h->Bm, ldb, ldb, h->Ysm, 16, 16, h->Ubuf, 16, 1.0, 0.0);
    }
    copy_cols(s, n, h->Bm, ldb, 16, h->Ucpl, 16);
    if (h->n_iso > 0) {
        iso_merge(s, h->n_iso, h->iso_idx, h->dshift, 1, h->theta, h->res, h->plan);
        gather_ritz(s, n, h->Ucpl, h->plan, h->Uritz);
    }
    return cyc;
}

// ---------------------------------------------------------------------------
// one iteration of Alg. 1 (device work; one host synchronisation inside the
// Lanczos restart test and one for the alternating maximisation)
// ---------------------------------------------------------------------------
void polish_dual(usbs_handle *h, double stag = 0.0);

// expansion cycles every tight eigen-solve runs before its convergence test counts: a
// start block that already holds converged eigenvectors of lower eigenvalues would
// otherwise pass the residual test before the Krylov expansion has found the top one
constexpr int kCertifyMinCycles = 2;

// consecutive null steps after which f at the centre is re-evaluated with the tight
// eigen-solve (an inexact eigen-solve can under-estimate f at an accepted centre, after
// which no candidate passes the descent test)
constexpr int kStallWindow = 25;

// relative change of the top Ritz value over one cycle below which the stall re-evaluation
// stops expanding.  The top Ritz value rises towards lambda_1 at a roughly linear rate (about
// 0.45 per cycle on a 4-regular graph with 10^6 vertices), so the error left is of the order
// of the last change: f is then known to about 1e-6 relative, well inside what the descent test
// resolves near the 1e-3 gap, while a residual test at the tight tolerance can take the
// whole restart allowance.  The certification of a final iterate keeps the residual test.
constexpr double kPolishStag = 1e-6;

// Master-QP reductions (App. B.2): Q11 = sum_k g_k g_k^T when do_q11, then G^T w_j.  With
// diagonal constraints only, G^T w goes through the weighted Gram of V (wgram: one sweep over
// the n rows instead of the m constraint rows, no svec rows formed); otherwise qp_gram forms
// g_k per constraint row.  Same output layout either way.
void qp_gram_w(usbs_handle *h, const double *V, int k, const double *const *ws, int nw, double *out, int do_q11,
               hipStream_t s, const RedScratch &rs) {
    const int d = k * (k + 1) / 2;
    if (!h->has_offc) {
        if (do_q11) qp_gram(s, rs, h->m, h->kptr, h->ti, h->tj, h->tv, V, 16, k, nullptr, 0, out, 1);
        wgram(s, rs, h->n, V, 16, k, h->dptr, h->dk, h->dv, ws, nw, out + (do_q11 ? d * (d + 1) / 2 : 0));
    } else {
        qp_gram(s, rs, h->m, h->kptr, h->ti, h->tj, h->tv, V, 16, k, ws, nw, out, do_q11);
    }
}
void qp_gram_w(usbs_handle *h, const double *V, int k, const double *const *ws, int nw, double *out, int do_q11) {
    qp_gram_w(h, V, k, ws, nw, out, do_q11, h->stream, h->rs);
}

// the side stream and its events, created on first use
void ensure_side(usbs_handle *h) {
    if (h->side) return;
    HIPCHK(hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&h->ev_side0, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&h->ev_side1, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&h->ev_side2, hipEventDisableTiming));
}

void iterate(usbs_handle *h) {
    hipStream_t s = h->stream;
    const int n = h->n, m = h->m, k = h->k, kc = h->kc, kp = h->kp, r = h->r;
    const int d = k * (k + 1) / 2;
    const usbs_params &prm = h->prm;
    // The reductions of the master QP (sum g g^T, G^T zbar, G^T y, G^T b; matrix-core and LDS
    // bound) run on the side stream beside V^T C V (HBM bound) on the handle's stream; then
    // V^T Psi of the sketch update, which needs V only, runs there while the master QP is
    // solved on one workgroup (the model update waits for it).
    ensure_side(h);
    HIPCHK(hipEventRecord(h->ev_side0, s));
    HIPCHK(hipStreamWaitEvent(h->side, h->ev_side0, 0));
    {
        const double *ws[3] = {h->zbar, h->y, h->b};
        qp_gram_w(h, h->V, k, ws, 3, h->raw, 1, h->side, h->rs_side);
        HIPCHK(hipEventRecord(h->ev_side2, h->side));
        if (h->sketch) tn_reduce_f(h->side, h->rs_side, n, h->V, 16, k, h->psi, r, r, h->VtPsi, r, 1.0);
        HIPCHK(hipEventRecord(h->ev_side1, h->side));
    }
    // V^T C V
    apply_C(h, h->V, 16, h->CV, 16, 16);
    tn_reduce(s, h->rs, n, h->V, 16, k, h->CV, 16, k, h->VCV, k, 1.0, 0.0);
    {
        const double *a[3] = {h->zbar, h->y, h->b}, *bb[3] = {h->zbar, h->zbar, h->zbar};
        dots(s, h->rs, m, a, bb, 3, h->sc + SC_ZZ);
    }
    HIPCHK(hipStreamWaitEvent(s, h->ev_side2, 0));
    // alternating maximisation over (X, nu) (eqs. small_quad_sdp, dual_slack_update)
    fill(s, m, 0.0, h->nu);
    IpmArgs ia{k, 1e-7, 1e-7, 100, 0};
    for (int pass = 0; pass < 50; ++pass) {
        if (pass > 0) {
            const double *ws[1] = {h->nu};
            qp_gram_w(h, h->V, k, ws, 1, h->Gy, 0);
            // G^T nu lands after the d*d block of Gy; copy into raw's 4th vector slot
            HIPCHK(hipMemcpyAsync(h->raw + d * (d + 1) / 2 + 3 * d, h->Gy, d * sizeof(double),
                                  hipMemcpyDeviceToDevice, s));
            const double *a[1] = {h->nu}, *bb[1] = {h->zbar};
            dots(s, h->rs, m, a, bb, 1, h->sc + SC_NUZ);
        }
        qp_finalize(s, k, h->raw, h->VCV, h->sc, pass > 0, h->qp);
        ia.warm = pass > 0;
        {
            ProfScope ps(h, USBS_PROF_IPM);
            ipm(s, ia, h->qp, h->ipm);
        }
        post_ipm(s, k, h->ipm, h->VCV, h->sc);
        // A X_{t+1} = g zbar + alpha A(V S V^T)
        lowrank_A(s, m, h->kptr, h->ti, h->tj, h->tv, h->V, 16, k, h->ipm, prm.alpha, h->zbar, h->sc + SC_G, 0.0,
                  h->AX, 0.0);
        if (!h->has_ineq) break;
        nu_update(s, m, h->b, h->AX, h->y, h->ineq, prm.rho, h->nu, h->dnu);
        const double *a[1] = {h->dnu}, *bb[1] = {h->dnu};
        dots(s, h->rs, m, a, bb, 1, h->sc + SC_DNU);
        double dn = 0.0;
        HIPCHK(hipMemcpyAsync(&dn, h->sc + SC_DNU, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (std::sqrt(dn) <= 1e-9) break;
    }
    // candidate (eq. dual_update) and primal infeasibility of X_{t+1}
    candidate(s, m, h->b, h->AX, h->y, h->ineq, prm.rho, h->yc, h->evec);
    {
        const double *a[3] = {h->b, h->yc, h->evec}, *bb[3] = {h->yc, h->zbar, h->evec};
        dots(s, h->rs, m, a, bb, 3, h->sc + SC_BY);   // SC_BY, SC_YZ, SC_DIST2 are consecutive
        const double *ws[1] = {h->yc};
        qp_gram_w(h, h->V, k, ws, 1, h->Gy, 0);
        fhat_prep(s, k, h->VCV, h->Gy, h->sc);
    }
    // eigen step at the candidate: the previous Ritz block with its last two columns
    // replaced by fresh random directions (the new top eigenvector need not lie in it)
    shift_operator(h, h->yc);
    copy_cols(s, n, h->Ucpl, 16, 14, h->Ubuf, 16);
    random_block_pad(s, n, 2, prm.seed + 7919ull * (uint64_t)(h->iters + 1), h->W, 8);
    const double tol_rest = prm.lanczos_tol_rest > 0.0 ? prm.lanczos_tol_rest : std::sqrt(prm.lanczos_tol);
    const int cyc = lanczos(h, h->Ubuf, kc, prm.lanczos_tol, tol_rest, prm.lanczos_max_restarts, true, 0, 14, true);
    const bool at_cap = cyc >= prm.lanczos_max_restarts;
    decide(s, h->theta, h->sc);
    cond_copy(s, m, h->sc + SC_DESC, h->yc, h->y);
    // model update
    HIPCHK(hipStreamWaitEvent(s, h->ev_side1, 0));
    model_update(s, k, kp, r, h->ipm, h->VCV, h->VtPsi, h->sc, h->Kc, h->Qp, h->sketch ? h->Hsk : nullptr);
    lowrank_A(s, m, h->kptr, h->ti, h->tj, h->tv, h->V, 16, k, h->Kc, 1.0, h->zbar, h->sc + SC_G, 0.0, h->zbar,
              0.0);
    if (h->sketch) nn_update_dev_beta(h, h->V, 16, k, h->Hsk, r, r, h->P, r);
    // V_{t+1} = orth([V Q_p, v_1..v_kc]) (eq. v_next_def)
    copy_cols(s, n, h->Uritz, 16, kc, h->Vn, 16);
    if (kp > 0 && kp <= 8) {
        // V Q_p (zero-padded to 8 columns) orthonormalised against the kc Ritz vectors
        pad_small(s, k, kp, h->Qp, kp, h->Qp8, 8);
        nn_update(s, n, h->V, 16, k, h->Qp8, 8, 8, h->W, 8, 1.0, 0.0);
        set_int(s, h->zdead, 16, 0);
        orth_fresh(h, h->Uritz, 16, kc, h->Vn + kc, 16, kp, h->zdead, h->Tscr, 8);
        fix_dead(s, n, h->zdead, kc, kp, h->Uritz, 16, h->Vn, 16);
    } else if (kp > 0) {
        nn_update(s, n, h->V, 16, k, h->Qp, kp, kp, h->Zp, 16, 1.0, 0.0);
        for (int pass = 0; pass < 2; ++pass) {
            tn_reduce(s, h->rs, n, h->Uritz, 16, kc, h->Zp, 16, kp, h->hz, kp, 1.0, 0.0);
            nn_update(s, n, h->Uritz, 16, kc, h->hz, kp, kp, h->Zp, 16, -1.0, 1.0);
        }
        set_int(s, h->zdead, 16, 0);
        cholqr2(h, h->Zp, 16, kp, h->W2, 16, h->Vn + kc, 16, h->zdead);
        fix_dead(s, n, h->zdead, kc, kp, h->Uritz, 16, h->Vn, 16);
    }
    std::swap(h->V, h->Vn);
    h->iters++;
    h->primal_at = h->iters;
    double desc = 0.0;
    HIPCHK(hipMemcpyAsync(&desc, h->sc + SC_DESC, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (h->conv_pending) {
        h->last_conv = *h->conv_host != 0;
        h->conv_pending = false;
    }
    if (at_cap && !h->last_conv) h->lz_unconverged++;
    h->null_run = desc != 0.0 ? 0 : h->null_run + 1;
    if (h->null_run >= kStallWindow) {
        polish_dual(h, kPolishStag);
        h->null_run = 0;
        h->recoveries++;
    }
}

// accurate f(y_t): Lanczos on C - A^* y_t from the current Ritz vectors with a tight
// tolerance; f and the relative gap are recomputed from it (the iterate is unchanged).
// stag > 0 also ends it once the top Ritz value has settled (see lanczos)
void polish_dual(usbs_handle *h, double stag) {
    hipStream_t s = h->stream;
    shift_operator(h, h->y);
    // start: the 12 leading Ritz vectors of the last candidate plus 4 random directions
    copy_cols(s, h->n, h->Ucpl, 16, 12, h->Ubuf, 16);
    random_block_pad(s, h->n, 4, h->prm.seed + 1000003ull * (uint64_t)(h->iters + 1), h->W, 8);
    lanczos(h, h->Ubuf, 1, h->prm.lanczos_tol_final, h->prm.lanczos_tol_final, 30, true, kCertifyMinCycles, 12, false, stag);
    recompute_f(s, h->theta, h->y, h->b, h->m, h->rs, h->sc, 1);
}

}  // namespace

// nn_update with beta read from the device scalar g (sketch update of Sec. 4:
// P <- g P + V (Kc V^T Psi)), one sweep over P (C = P has exactly cc = ldc columns)
void nn_update_dev_beta(usbs_handle *h, const double *A, int lda, int ca, const double *H, int ldh, int cc, double *C,
                        int ldc) {
    nn_update_beta_dev(h->stream, h->n, A, lda, ca, H, ldh, cc, C, ldc, h->sc + SC_G);
}

namespace {

void init_scalars(usbs_handle *h) {
    std::vector<double> sc(SC_COUNT, 0.0);
    sc[SC_BNORM] = h->bnorm;
    sc[SC_SIGMA] = h->sigma;
    sc[SC_TRACE] = h->trace;
    sc[SC_ALPHA] = h->prm.alpha;
    sc[SC_RHO] = h->prm.rho;
    sc[SC_BETA] = h->prm.beta;
    sc[SC_UNITS] = h->prm.units;
    HIPCHK(hipMemcpyAsync(h->sc, sc.data(), SC_COUNT * sizeof(double), hipMemcpyHostToDevice, h->stream));
}

// cold start (reading of Alg. 1's unspecified initialisation): y0 = 0,
// V0 = top-k eigenvectors of C_s, Xbar0 = 0, f0 = f(y0)
void cold_start(usbs_handle *h) {
    hipStream_t s = h->stream;
    HIPCHK(hipMemsetAsync(h->y, 0, h->m * sizeof(double), s));
    HIPCHK(hipMemsetAsync(h->zbar, 0, h->m * sizeof(double), s));
    HIPCHK(hipMemsetAsync(h->P, 0, (size_t)h->n * std::max(h->r, 1) * sizeof(double), s));
    init_scalars(h);
    random_block(s, h->n, 16, h->prm.seed, h->Ubuf, 16);
    shift_operator(h, h->y);
    lanczos(h, h->Ubuf, h->k, h->prm.lanczos_tol_final, std::sqrt(h->prm.lanczos_tol_final),
            std::max(h->prm.lanczos_max_restarts, 30), true, kCertifyMinCycles);
    HIPCHK(hipMemsetAsync(h->V, 0, (size_t)h->n * 16 * sizeof(double), s));
    copy_cols(s, h->n, h->Uritz, 16, h->k, h->V, 16);
    // f(y0) = alpha [theta_1]_+ (b^T y0 = 0)
    std::vector<double> th(1);
    HIPCHK(hipMemcpyAsync(th.data(), h->theta, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const double f0 = h->prm.alpha * std::max(th[0], 0.0);
    HIPCHK(hipMemcpyAsync(h->sc + SC_F, &f0, sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
}

void check_params(const usbs_params *p) {
    if (!p) throw DevError(USBS_E_INVALID, "params is NULL");
    if (!(p->alpha > 0) || !(p->rho > 0) || !(p->beta > 0 && p->beta < 1))
        throw DevError(USBS_E_INVALID, "need alpha > 0, rho > 0, 0 < beta < 1");
    if (p->k_c < 1 || p->k_p < 0 || p->k_c + p->k_p > kMaxK)
        throw DevError(USBS_E_INVALID, "need k_c >= 1, k_p >= 0, k_c + k_p <= 12");
    if (p->k_c + p->k_p > kRitz - 2) throw DevError(USBS_E_INVALID, "k_c + k_p too large for the Ritz block");
    if (p->r < 0 || p->r > kMaxRank) throw DevError(USBS_E_INVALID, "need 0 <= r <= 16");
    if (p->lanczos_steps < 1 || p->lanczos_steps > kMaxSteps)
        throw DevError(USBS_E_INVALID, "need 1 <= lanczos_steps <= 8");
    if (p->lanczos_max_restarts < 0) throw DevError(USBS_E_INVALID, "lanczos_max_restarts < 0");
    if (!(p->lanczos_tol > 0) || !(p->lanczos_tol_final > 0)) throw DevError(USBS_E_INVALID, "Lanczos tolerances must be > 0");
    if (p->precision < 0 || p->precision > 2) throw DevError(USBS_E_INVALID, "unknown precision");
    if (p->units != USBS_UNITS_SCALED && p->units != USBS_UNITS_ORIGINAL)
        throw DevError(USBS_E_INVALID, "unknown units");
    if (p->autotune < 0 || p->autotune > 2) throw DevError(USBS_E_INVALID, "autotune must be 0, 1 or 2");
}

// ---------------------------------------------------------------------------
// autotuner: times the candidate launch shapes of the tuned kernels on the handle's own
// buffers and shapes (hipEvents on its stream, best of three after a warm-up launch)
// and keeps the fastest; results are cached per (device, log2 n, log2 nonzeros per row,
// precision, mode) for the life of the process
// ---------------------------------------------------------------------------
struct TuneKey {
    int dev, nb, zb, prec, mode;
    bool operator<(const TuneKey &o) const {
        return std::tie(dev, nb, zb, prec, mode) < std::tie(o.dev, o.nb, o.zb, o.prec, o.mode);
    }
};
std::mutex g_tune_mu;
std::map<TuneKey, Tuning> g_tune_cache;

template <typename F>
float time_launch(hipStream_t s, F &&launch) {
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    launch();
    float best = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {
        HIPCHK(hipEventRecord(e0, s));
        launch();
        HIPCHK(hipEventRecord(e1, s));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        best = std::min(best, ms);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return best;
}

void autotune(usbs_handle *h) {
    h->tune = Tuning{};
    const int mode = h->prm.autotune;
    if (mode == 0) return;
    const int n = h->n;
    auto lg = [](double v) { int b = 0; while (v >= 2.0) { v *= 0.5; ++b; } return b; };
    const TuneKey key{h->dev, lg(n), lg(1.0 + (double)h->nnz / std::max(n, 1)), h->prec, mode};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            h->tune = it->second;
            return;
        }
    }
    hipStream_t s = h->stream;
    const int ldb = h->ldb, cols = ldb - 8;
    Tuning t;
    set_tuning(&t);
    // SpMM with 8 and 16 columns: 1, 2 or 4 columns per lane
    for (int nb : {8, 16}) {
        float best = 1e30f;
        int arg = 0;
        for (int var = 0; var < 3; ++var) {
            (nb == 8 ? t.spmm8 : t.spmm16) = var;
            const float ms = time_launch(s, [&] {
                spmm(s, h->prec, n, h->rowptr, h->col, h->val_cur, h->val_scale, h->dshift, h->Bm, ldb,
                     nb == 8 ? h->W : h->Ubuf, nb == 8 ? 8 : 16, nb);
            });
            if (ms < best) {
                best = ms;
                arg = var;
            }
        }
        (nb == 8 ? t.spmm8 : t.spmm16) = arg;
    }
    // grid cap of the MFMA update ([Q W] coef as in a Lanczos block step)
    {
        float best = 1e30f;
        int arg = 4096;
        for (int cap : {1024, 2048, 4096, 8192}) {
            t.nn_cap = cap;
            const float ms = time_launch(s, [&] {
                nn_update2(s, n, h->Bm, ldb, cols, h->W, 8, 8, h->coef, 8, 8, h->Wt, 8);
            });
            if (ms < best) {
                best = ms;
                arg = cap;
            }
        }
        t.nn_cap = arg;
    }
    // partition of the matrix-core reductions (changes rounding: only on request)
    if (mode == 2) {
        float best = 1e30f;
        int bc = 512, bu = 4;
        for (int cap : {128, 256, 512})
            for (int unr : {2, 4}) {
                t.red_cap = cap;
                t.red_unr = unr;
                const float ms = time_launch(s, [&] { reorth_partials(s, h->rs, n, h->Bm, ldb, cols, h->W, 8, 8); });
                if (ms < best) {
                    best = ms;
                    bc = cap;
                    bu = unr;
                }
            }
        t.red_cap = bc;
        t.red_unr = bu;
    }
    set_tuning(nullptr);
    h->tune = t;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = t;
}

// the handle's launch shapes for every kernel launched from this thread during a call
struct TuneScope {
    explicit TuneScope(const usbs_handle *h) { set_tuning(h ? &h->tune : nullptr); }
    ~TuneScope() { set_tuning(nullptr); }
};

void configure(usbs_handle *h, const usbs_params *p) {
    h->prm = *p;
    h->kc = p->k_c;
    h->kp = p->k_p;
    h->k = p->k_c + p->k_p;
    h->r = p->r;
    h->prec = p->precision;
    h->stream = (hipStream_t)p->stream;
}

void set_geometry(usbs_handle *h, int n) {
    // the basis (16 + 8 s columns) must stay well inside R^n
    int steps = h->prm.lanczos_steps;
    while (steps > 1 && 2 * (16 + 8 * steps) > n) --steps;
    if (2 * (16 + 8) > n) throw DevError(USBS_E_INVALID, "n too small for the block Lanczos basis (need n >= 48)");
    h->steps = steps;
    h->ldb = 16 + 8 * steps;
}

int fail(usbs_handle *h, const DevError &e) {
    set_err(h, e.what());
    return e.code;
}

}  // namespace

namespace {
// Results of a finished solve (usbs_result, y in original units, Nystrom factors of the
// sketch and their certificate terms) from the device state of the handle.
void fill_result(usbs_handle *h, usbs_result *res, double *y_out, double *U_out, double *lam_out, int status, int it,
                 double secs) {
    const usbs_params &p = h->prm;
    std::vector<double> sc(SC_COUNT);
    HIPCHK(hipMemcpyAsync(sc.data(), h->sc, SC_COUNT * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    if (res) {
        std::memset(res, 0, sizeof(*res));
        const double s = h->sigma * h->trace;
        res->primal_obj_scaled = sc[SC_CX];
        res->f_scaled = sc[SC_F];
        res->primal_obj = s * sc[SC_CX];
        res->dual_bound = s * sc[SC_F];
        res->rel_gap = sc[SC_GAP];
        res->rel_infeas = sc[SC_INF];
        {
            const double s2 = h->sigma * h->trace, dist = std::sqrt(std::max(sc[SC_DIST2], 0.0));
            res->rel_gap_scaled = std::fabs(sc[SC_F] - sc[SC_CX]) / (1.0 + std::fabs(sc[SC_CX]));
            res->rel_infeas_scaled = dist / (1.0 + h->bnorm);
            res->rel_gap_original = std::fabs(s2 * sc[SC_F] - s2 * sc[SC_CX]) / (1.0 + std::fabs(s2 * sc[SC_CX]));
            res->rel_infeas_original = h->trace * dist / (1.0 + h->trace * h->bnorm);
        }
        res->lanczos_unconverged = h->lz_unconverged;
        res->stall_recoveries = h->recoveries;
        res->lambda_max = sc[SC_THETA1];
        res->seconds = secs;
        res->lanczos_matvecs = h->matvecs;
        res->iters = it;
        res->descents = (int)sc[SC_NDESC];
        res->ipm_iters = (int)sc[SC_IPMIT];
        res->status = status;
    }
    if (y_out) {
        std::vector<double> yv(h->m);
        HIPCHK(hipMemcpyAsync(yv.data(), h->y, h->m * sizeof(double), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        for (int q = 0; q < h->m; ++q) y_out[q] = h->sigma * yv[q];
    }
    if ((U_out || lam_out || res) && h->sketch && h->r > 0) {
        // Nystrom reconstruction of Xbar (App. C.1) and its certificate terms
        const int n = h->n, r = h->r;
        hipStream_t s = h->stream;
        interleave(s, n, r, h->P, h->psi, h->W2);
        tn_reduce(s, h->rs, n, h->W2, 2 * r, 2 * r, h->W2, 2 * r, 2 * r, h->small, 2 * r, 1.0, 0.0);
        nystrom_core(s, n, r, h->small, h->small + 1024, h->small + 2048, h->flag);
        nn_update(s, n, h->W2, 2 * r, 2 * r, h->small + 1024, r, r, h->Zp, 16, 1.0, 0.0);
        std::vector<double> lam(r);
        HIPCHK(hipMemcpyAsync(lam.data(), h->small + 2048, r * sizeof(double), hipMemcpyDeviceToHost, s));
        // <C_s, Xhat> = sum_j lam_j u_j^T C_s u_j ; A(Xhat)
        apply_C(h, h->Zp, 16, h->CV, 16, r);
        tn_reduce(s, h->rs, n, h->Zp, 16, r, h->CV, 16, r, h->TUU, r, 1.0, 0.0);
        std::vector<double> uc(r * r);
        HIPCHK(hipMemcpyAsync(uc.data(), h->TUU, r * r * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        double cx = 0.0;
        for (int j = 0; j < r; ++j) cx += lam[j] * uc[j * r + j];
        std::vector<double> K(r * r, 0.0);
        for (int j = 0; j < r; ++j) K[j * r + j] = lam[j];
        HIPCHK(hipMemcpyAsync(h->Kc, K.data(), r * r * sizeof(double), hipMemcpyHostToDevice, s));
        // A(Xhat) goes to its own buffer: AX keeps A X_{t+1} for usbs_get_primal
        lowrank_A(s, h->m, h->kptr, h->ti, h->tj, h->tv, h->Zp, 16, r, h->Kc, 1.0, nullptr, nullptr, 0.0, h->AXhat,
                  0.0);
        std::vector<double> ax(h->m), bs(h->m);
        HIPCHK(hipMemcpyAsync(ax.data(), h->AXhat, h->m * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(bs.data(), h->b, h->m * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        double d2 = 0.0;
        for (int q = 0; q < h->m; ++q) {
            const double e = h->hp.ineq[q] ? std::max(ax[q] - bs[q], 0.0) : ax[q] - bs[q];
            d2 += e * e;
        }
        if (res) {
            res->sketch_primal_obj = h->sigma * h->trace * cx;
            res->sketch_rel_infeas = (p.units == USBS_UNITS_ORIGINAL)
                                         ? h->trace * std::sqrt(d2) / (1.0 + h->trace * h->bnorm)
                                         : std::sqrt(d2) / (1.0 + h->bnorm);
        }
        if (lam_out)
            for (int j = 0; j < r; ++j) lam_out[j] = h->trace * lam[j];
        if (U_out) {
            std::vector<double> U((size_t)n * 16);
            HIPCHK(hipMemcpyAsync(U.data(), h->Zp, (size_t)n * 16 * sizeof(double), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < r; ++j) U_out[(size_t)i * r + j] = U[(size_t)i * 16 + j];
        }
    }
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int usbs_default_params(usbs_params *p) {
    if (!p) return USBS_E_INVALID;
    std::memset(p, 0, sizeof(*p));
    p->alpha = 2.0;
    p->rho = 0.01;
    p->beta = 0.25;
    p->k_c = 10;
    p->k_p = 1;
    p->r = 10;
    p->eps_gap = 1e-3;
    p->eps_infeas = 1e-3;
    p->units = USBS_UNITS_SCALED;
    p->max_iters = 1000;
    p->time_limit = 0.0;
    p->lanczos_steps = 8;   // 64 new Krylov vectors per restart cycle (block 8)
    p->lanczos_max_restarts = 10;   // the paper's restart limit
    p->lanczos_tol = 1e-4;
    p->lanczos_tol_final = 1e-9;
    p->precision = USBS_PREC_F64;
    p->seed = 0;
    p->stream = nullptr;
    p->verbose = 0;
    p->autotune = 1;
    p->lanczos_tol_rest = 0.0;
    return USBS_OK;
}

int usbs_create(const usbs_problem *prob, const usbs_params *prm, usbs_handle **out) {
    return usbs_pack::create(prob, prm, out, true);
}

}  // extern "C"

namespace usbs_pack {
// usbs_create; with cold = false the cold start is left to the packed kernel
// (PACK_INIT_COLD): the scalars are initialised and the work arrays cleared here
int create(const usbs_problem *prob, const usbs_params *prm, usbs_handle **out, bool cold) {
    if (!out) return USBS_E_INVALID;
    *out = nullptr;
    usbs_handle *h = new usbs_handle();
    try {
        check_params(prm);
        configure(h, prm);
        HIPCHK(hipGetDevice(&h->dev));
        h->hp = copy_problem(prob, h->r);
        if (h->hp.psi.empty() && !h->prm.psi_from_seed) h->r = 0;
        set_geometry(h, h->hp.n);
        upload(h);
        if (cold) {
            autotune(h);
            TuneScope tsc(h);
            cold_start(h);
        } else {
            init_scalars(h);
            HIPCHK(hipStreamSynchronize(h->stream));
        }
        h->ready = true;
    } catch (const DevError &e) {
        *out = h;   // the handle carries the message; caller frees it
        const int c = fail(h, e);
        free_problem(h);
        h->ready = false;
        return c;
    }
    *out = h;
    return USBS_OK;
}
}  // namespace usbs_pack

extern "C" {

int usbs_solve(usbs_handle *h, usbs_result *res, double *y_out, double *U_out, double *lam_out) {
    if (!h || !h->ready) {
        set_err(h, "handle not ready");
        return USBS_E_STATE;
    }
    try {
        TuneScope tsc(h);
        const auto t0 = std::chrono::steady_clock::now();
        const usbs_params &p = h->prm;
        std::vector<double> sc(SC_COUNT);
        int status = USBS_NOT_CONVERGED;
        int it = 0;
        for (it = 0; it < p.max_iters; ++it) {
            iterate(h);
            HIPCHK(hipMemcpyAsync(sc.data(), h->sc, SC_COUNT * sizeof(double), hipMemcpyDeviceToHost, h->stream));
            HIPCHK(hipStreamSynchronize(h->stream));
            if (!std::isfinite(sc[SC_F]) || !std::isfinite(sc[SC_CX]) || sc[SC_IPMSTATUS] == 2.0)
                throw DevError(USBS_E_NUMERIC, "non-finite iterate or failed interior point solve");
            if (p.verbose)
                std::fprintf(stderr, "it %d f %.8e fc %.8e fhat %.8e desc %d gap %.3e inf %.3e cX %.8e mv %lld\n",
                             h->iters, sc[SC_F], sc[SC_FCAND], sc[SC_FHAT], (int)sc[SC_DESC], sc[SC_GAP], sc[SC_INF],
                             sc[SC_CX], (long long)h->matvecs);
            if (sc[SC_GAP] <= p.eps_gap && sc[SC_INF] <= p.eps_infeas) {
                // certify: recompute lambda_max(C - A^* y_T) with a tight residual tolerance
                // so that the reported f(y_T) is an accurate upper bound, then re-test
                polish_dual(h);
                HIPCHK(hipMemcpyAsync(sc.data(), h->sc, SC_COUNT * sizeof(double), hipMemcpyDeviceToHost,
                                      h->stream));
                HIPCHK(hipStreamSynchronize(h->stream));
                if (sc[SC_GAP] <= p.eps_gap && sc[SC_INF] <= p.eps_infeas) {
                    status = USBS_OK;
                    ++it;
                    break;
                }
            }
            const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            if (p.time_limit > 0.0 && el > p.time_limit) {
                ++it;
                break;
            }
        }
        if (status != USBS_OK) {
            // stopped by a limit: report f(y_T) from the tight eigen-solve as well
            polish_dual(h);
            HIPCHK(hipMemcpyAsync(sc.data(), h->sc, SC_COUNT * sizeof(double), hipMemcpyDeviceToHost, h->stream));
            HIPCHK(hipStreamSynchronize(h->stream));
        }
        const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        fill_result(h, res, y_out, U_out, lam_out, status, it, secs);
        return status;
    } catch (const DevError &e) {
        return fail(h, e);
    }
}

void usbs_free(usbs_handle *h) {
    if (!h) return;
    if (h->side) (void)hipStreamSynchronize(h->side);
    free_problem(h);
    if (h->ev_side0) (void)hipEventDestroy(h->ev_side0);
    if (h->ev_side1) (void)hipEventDestroy(h->ev_side1);
    if (h->ev_side2) (void)hipEventDestroy(h->ev_side2);
    if (h->side) (void)hipStreamDestroy(h->side);
    if (h->conv_host) (void)hipHostFree(h->conv_host);
    for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
    delete h;
}

int usbs_profile(usbs_handle *h, int32_t category, int32_t reset, double *ms_total, int64_t *launches) {
    if (!h || !h->ready) return USBS_E_STATE;
    if (category < -1 || category >= USBS_PROF_COUNT) {
        set_err(h, "usbs_profile: unknown category");
        return USBS_E_INVALID;
    }
    try {
        if (h->ev_pool.empty() && category >= 0) {
            h->ev_pool.resize(8192);
            for (auto &e : h->ev_pool) HIPCHK(hipEventCreate(&e));
        }
        prof_flush(h);
        if (ms_total) *ms_total = h->prof_ms;
        if (launches) *launches = h->prof_count;
        if (reset) {
            h->prof_ms = 0.0;
            h->prof_count = 0;
        }
        h->prof_cat = category;
        return USBS_OK;
    } catch (const DevError &e) {
        return fail(h, e);
    }
}

const char *usbs_last_error(const usbs_handle *h) {
    if (h) return h->err.c_str();
    const char *m = usbs_noalloc::last_error();
    return m ? m : "NULL handle";
}

int64_t usbs_footprint_bytes(const usbs_problem *p, const usbs_params *prm) {
    if (!p || !prm || p->n < 1 || p->m < 1 || !p->rowptr || (p->n_triplets > 0 && (!p->a_i || !p->a_j)))
        return -1;
    const int64_t n = p->n, m = p->m, nt = p->n_triplets;
    const int64_t nnzC = p->rowptr[n];
    if (nnzC < 0) return -1;
    int64_t offt = 0;
    for (int64_t t = 0; t < nt; ++t) offt += (p->a_i[t] != p->a_j[t]);
    const int64_t diagt = nt - offt;
    const int64_t nnz = nnzC + 2 * offt;   // bound on the off-diagonal pattern
    const int64_t vsz = prm->precision == USBS_PREC_F64 ? 8 : (prm->precision == USBS_PREC_F32 ? 4 : 2);
    const int64_t r = (p->psi || prm->psi_from_seed) ? std::max(prm->r, 0) : 0;
    int64_t b = 0;
    // operator and constraints
    b += 4 * (n + 1) + 4 * nnz + 8 * nnz + 2 * vsz * nnz + 8 * 2 * n + 4 * (n + 1);
    b += 12 * diagt + 16 * 2 * offt + 4 * (m + 1) + 16 * nt + 16 * m + 4 * n * r;
    // iteration state and Lanczos work (see upload)
    b += 8 * 8 * m;
    b += 8 * n * 16 * 7;                       // V, Vn, CV, Uritz, Ucpl, Ubuf, Zp
    b += 8 * n * std::max<int64_t>(r, 1);     // sketch
    b += 8 * n * kMaxBasis + 8 * n * 8 * 2 + 8 * n * 32;
    // reduction partials and small matrices
    const int64_t max_elems = std::max<int64_t>(kMaxSvec * (kMaxSvec + 1) / 2 + 4 * kMaxSvec, kMaxBasis * 16);
    b += 8 * (int64_t)kRedMaxBlocks * max_elems;
    b += 8 * (4096 + 6 * 1024 + 8 * kMaxSvec * kMaxSvec) + 4 * 256;
    return b + b / 20 + (1 << 20);   // allocator rounding
}

int usbs_get_tuning(const usbs_handle *h, int32_t *out) {
    if (!h || !out) return USBS_E_INVALID;
    out[0] = h->tune.spmm8;
    out[1] = h->tune.spmm16;
    out[2] = h->tune.nn_cap;
    out[3] = h->tune.red_cap;
    out[4] = h->tune.red_unr;
    return USBS_OK;
}

int usbs_get_scaling(const usbs_handle *h, double *sigma, double *trace) {
    if (!h || !h->ready) return USBS_E_STATE;
    if (sigma) *sigma = h->sigma;
    if (trace) *trace = h->trace;
    return USBS_OK;
}

int usbs_op_apply(usbs_handle *h, const double *y_dev, const double *X_dev, int32_t ldx, double *Y_dev, int32_t ldy,
                  int32_t nb) {
    if (!h || !h->ready) return USBS_E_STATE;
    if (!y_dev || !X_dev || !Y_dev || nb < 1 || nb > 16 || ldx < nb || ldy < nb) {
        set_err(h, "usbs_op_apply: bad arguments");
        return USBS_E_INVALID;
    }
    try {
        TuneScope tsc(h);
        shift_operator(h, y_dev);
        apply_op(h, X_dev, ldx, Y_dev, ldy, nb);
        HIPCHK(hipStreamSynchronize(h->stream));
        return USBS_OK;
    } catch (const DevError &e) {
        return fail(h, e);
    }
}

int usbs_op_eigs(usbs_handle *h, const double *y_dev, int32_t k, const double *start_dev, double *w, double *U_dev,
                 double *res, int32_t *cycles) {
    if (!h || !h->ready) return USBS_E_STATE;
    if (!y_dev || k < 1 || k > 14) {
        set_err(h, "usbs_op_eigs: need y_dev and 1 <= k <= 14");
        return USBS_E_INVALID;
    }
    try {
        TuneScope tsc(h);
        hipStream_t s = h->stream;
        shift_operator(h, y_dev);
        if (start_dev) copy_cols(s, h->n, start_dev, 16, 16, h->Ubuf, 16);
        else random_block(s, h->n, 16, h->prm.seed + 7, h->Ubuf, 16);
        const int c = lanczos(h, h->Ubuf, k, h->prm.lanczos_tol_final, h->prm.lanczos_tol_final,
                              std::max(h->prm.lanczos_max_restarts, 30), true, kCertifyMinCycles);
        if (w) HIPCHK(hipMemcpyAsync(w, h->theta, k * sizeof(double), hipMemcpyDeviceToHost, s));
        if (res) HIPCHK(hipMemcpyAsync(res, h->res, k * sizeof(double), hipMemcpyDeviceToHost, s));
        if (U_dev) copy_cols(s, h->n, h->Uritz, 16, 16, U_dev, 16);
        HIPCHK(hipStreamSynchronize(s));
        if (cycles) *cycles = c;
        return USBS_OK;
    } catch (const DevError &e) {
        return fail(h, e);
    }
}

int usbs_op_lowrank_A(usbs_handle *h, const double *W_dev, int32_t q, const double *lam, double *out_dev) {
    if (!h || !h->ready) return USBS_E_STATE;
    if (!W_dev || !lam || !out_dev || q < 1 || q > 16) {
        set_err(h, "usbs_op_lowrank_A: bad arguments");
        return USBS_E_INVALID;
    }
    try {
        TuneScope tsc(h);
        std::vector<double> K(q * q, 0.0);
        for (int j = 0; j < q; ++j) K[j * q + j] = lam[j];
        HIPCHK(hipMemcpyAsync(h->Kc, K.data(), q * q * sizeof(double), hipMemcpyHostToDevice, h->stream));
        lowrank_A(h->stream, h->m, h->kptr, h->ti, h->tj, h->tv, W_dev, q, q, h->Kc, 1.0, nullptr, nullptr, 0.0,
                  out_dev, 0.0);
        HIPCHK(hipStreamSynchronize(h->stream));
        return USBS_OK;
    } catch (const DevError &e) {
        return fail(h, e);
    }
}

int usbs_op_sketch_update(usbs_handle *h, double g, const double *W_dev, int32_t q, const double *lam, double *P_dev) {
    if (!h || !h->ready) return USBS_E_STATE;
    if (!h->sketch) {
        set_err(h, "usbs_op_sketch_update: problem has no test matrix");
        return USBS_E_STATE;
    }
    if (!W_dev || !lam || !P_dev || q < 1 || q > 16) {
        set_err(h, "usbs_op_sketch_update: bad arguments");
        return USBS_E_INVALID;
    }
    try {
        TuneScope tsc(h);
        hipStream_t s = h->stream;
        const int r = h->r;
        tn_reduce_f(s, h->rs, h->n, W_dev, q, q, h->psi, r, r, h->VtPsi, r, 1.0);
        std::vector<double> G(q * r);
        HIPCHK(hipMemcpyAsync(G.data(), h->VtPsi, q * r * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (int a = 0; a < q; ++a)
            for (int c = 0; c < r; ++c) G[a * r + c] *= lam[a];
        HIPCHK(hipMemcpyAsync(h->Hsk, G.data(), q * r * sizeof(double), hipMemcpyHostToDevice, s));
        nn_update(s, h->n, W_dev, q, q, h->Hsk, r, r, P_dev, r, 1.0, g);
        HIPCHK(hipStreamSynchronize(s));
        return USBS_OK;
    } catch (const DevError &e) {
        return fail(h, e);
    }
}

int usbs_op_qp_data(usbs_handle *h, const double *V_dev, int32_t k, const double *y_dev, const double *w_dev,
                    const double *zbar_dev, double tau, double cbar, double *Q11, double *q12, double *q22,
                    double *h1, double *h2) {
    if (!h || !h->ready) return USBS_E_STATE;
    if (!V_dev || !y_dev || !w_dev || !zbar_dev || k < 1 || k > kMaxK) {
        set_err(h, "usbs_op_qp_data: bad arguments");
        return USBS_E_INVALID;
    }
    try {
        TuneScope tsc(h);
        hipStream_t s = h->stream;
        const int n = h->n, m = h->m, d = k * (k + 1) / 2;
        copy_cols(s, n, V_dev, k, k, h->Zp, 16);
        apply_C(h, h->Zp, 16, h->CV, 16, k);
        tn_reduce(s, h->rs, n, h->Zp, 16, k, h->CV, 16, k, h->VCV, k, 1.0, 0.0);
        const double *ws[3] = {zbar_dev, y_dev, w_dev};
        qp_gram_w(h, h->Zp, k, ws, 3, h->raw, 1);
        const double *a[3] = {zbar_dev, y_dev, w_dev}, *bb[3] = {zbar_dev, zbar_dev, zbar_dev};
        std::vector<double> sc(SC_COUNT, 0.0);
        HIPCHK(hipMemcpyAsync(sc.data(), h->sc, SC_COUNT * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        std::vector<double> save = sc;
        sc[SC_TAU] = tau;
        sc[SC_CBAR] = cbar;
        HIPCHK(hipMemcpyAsync(h->sc, sc.data(), SC_COUNT * sizeof(double), hipMemcpyHostToDevice, s));
        dots(s, h->rs, m, a, bb, 3, h->sc + SC_ZZ);
        qp_finalize(s, k, h->raw, h->VCV, h->sc, 0, h->qp);
        std::vector<double> out(d * d + 2 * d + 2);
        HIPCHK(hipMemcpyAsync(out.data(), h->qp, out.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        HIPCHK(hipMemcpyAsync(h->sc, save.data(), SC_COUNT * sizeof(double), hipMemcpyHostToDevice, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        if (Q11) std::memcpy(Q11, out.data(), d * d * sizeof(double));
        if (q12) std::memcpy(q12, out.data() + d * d, d * sizeof(double));
        if (q22) *q22 = out[d * d + d];
        if (h1) std::memcpy(h1, out.data() + d * d + d + 1, d * sizeof(double));
        if (h2) *h2 = out[d * d + 2 * d + 1];
        return USBS_OK;
    } catch (const DevError &e) {
        return fail(h, e);
    }
}

int usbs_op_ipm(usbs_handle *h, int32_t k, const double *Q11, const double *q12, double q22, const double *h1,
                double h2, double *S, double *eta, int32_t *iters) {
    if (!h || !h->ready) return USBS_E_STATE;
    if (k < 1 || k > kMaxK || !Q11 || !q12 || !h1) {
        set_err(h, "usbs_op_ipm: bad arguments");
        return USBS_E_INVALID;
    }
    try {
        TuneScope tsc(h);
        hipStream_t s = h->stream;
        const int d = k * (k + 1) / 2;
        std::vector<double> qpv(d * d + 2 * d + 2);
        std::memcpy(qpv.data(), Q11, d * d * sizeof(double));
        std::memcpy(qpv.data() + d * d, q12, d * sizeof(double));
        qpv[d * d + d] = q22;
        std::memcpy(qpv.data() + d * d + d + 1, h1, d * sizeof(double));
        qpv[d * d + 2 * d + 1] = h2;
        HIPCHK(hipMemcpyAsync(h->qp, qpv.data(), qpv.size() * sizeof(double), hipMemcpyHostToDevice, s));
        IpmArgs ia{k, 1e-7, 1e-7, 100, 0};
        ipm(s, ia, h->qp, h->ipm);
        std::vector<double> st(2 * k * k + 5);
        HIPCHK(hipMemcpyAsync(st.data(), h->ipm, st.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (S) std::memcpy(S, st.data(), k * k * sizeof(double));
        if (eta) *eta = st[2 * k * k];
        if (iters) *iters = (int)st[2 * k * k + 3];
        if (st[2 * k * k + 4] == 2.0) {
            set_err(h, "interior point method failed (numerical breakdown)");
            return USBS_E_NUMERIC;
        }
        return USBS_OK;
    } catch (const DevError &e) {
        return fail(h, e);
    }
}

int usbs_op_nystrom(usbs_handle *h, const double *P_dev, double *U_dev, double *lam) {
    if (!h || !h->ready) return USBS_E_STATE;
    if (!h->sketch || !P_dev || !U_dev) {
        set_err(h, "usbs_op_nystrom: needs a test matrix and device arrays");
        return USBS_E_INVALID;
    }
    try {
        TuneScope tsc(h);
        hipStream_t s = h->stream;
        const int n = h->n, r = h->r;
        interleave(s, n, r, P_dev, h->psi, h->W2);
        tn_reduce(s, h->rs, n, h->W2, 2 * r, 2 * r, h->W2, 2 * r, 2 * r, h->small, 2 * r, 1.0, 0.0);
        nystrom_core(s, n, r, h->small, h->small + 1024, h->small + 2048, h->flag);
        nn_update(s, n, h->W2, 2 * r, 2 * r, h->small + 1024, r, r, U_dev, r, 1.0, 0.0);
        int bad = 0;
        if (lam) HIPCHK(hipMemcpyAsync(lam, h->small + 2048, r * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(&bad, h->flag, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (bad) {
            set_err(h, "Nystrom core matrix not positive definite");
            return USBS_E_NUMERIC;
        }
        return USBS_OK;
    } catch (const DevError &e) {
        return fail(h, e);
    }
}

int usbs_round_maxcut(usbs_handle *h, int8_t *x_out, double *cut_out, int32_t *column_out, double *cuts_out) {
    if (!h || !h->ready) return USBS_E_STATE;
    if (!h->sketch || h->r < 1) {
        set_err(h, "usbs_round_maxcut: needs the Nystrom sketch (r > 0 and a test matrix)");
        return USBS_E_INVALID;
    }
    try {
        TuneScope tsc(h);
        hipStream_t s = h->stream;
        const int n = h->n, r = h->r;
        // U of the Nystrom reconstruction of the current sketch (App. C.1)
        interleave(s, n, r, h->P, h->psi, h->W2);
        tn_reduce(s, h->rs, n, h->W2, 2 * r, 2 * r, h->W2, 2 * r, 2 * r, h->small, 2 * r, 1.0, 0.0);
        nystrom_core(s, n, r, h->small, h->small + 1024, h->small + 2048, h->flag);
        nn_update(s, n, h->W2, 2 * r, 2 * r, h->small + 1024, r, r, h->Zp, 16, 1.0, 0.0);
        // x_c^T C x_c for the r sign vectors, FP64 (the base values, not the compute copy)
        quad_forms(s, h->rs, n, r, h->rowptr, h->col, h->cbase, h->cdiag, h->Zp, 16, h->Ubuf, h->small + 3072);
        std::vector<double> q(r);
        int bad = 0;
        HIPCHK(hipMemcpyAsync(q.data(), h->small + 3072, r * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(&bad, h->flag, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (bad) throw DevError(USBS_E_NUMERIC, "Nystrom core matrix not positive definite");
        int best = 0;
        for (int c = 1; c < r; ++c)
            if (q[c] > q[best]) best = c;   // first of equal values
        if (cut_out) *cut_out = h->sigma * q[best];
        if (column_out) *column_out = best;
        if (cuts_out)
            for (int c = 0; c < r; ++c) cuts_out[c] = h->sigma * q[c];
        if (x_out) {
            std::vector<double> S((size_t)n * 16);
            HIPCHK(hipMemcpyAsync(S.data(), h->Ubuf, (size_t)n * 16 * sizeof(double), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            for (int i = 0; i < n; ++i) x_out[i] = S[(size_t)i * 16 + best] > 0.0 ? 1 : -1;
        }
        return USBS_OK;
    } catch (const DevError &e) {
        return fail(h, e);
    }
}

int usbs_step_iterate(usbs_handle *h, int32_t t, double *y, double *V, double *zbar, double *Pbar, double *scal) {
    if (!h || !h->ready) return USBS_E_STATE;
    if (t < 0) return USBS_E_INVALID;
    try {
        TuneScope tsc(h);
        for (int q = 0; q < t; ++q) iterate(h);
        hipStream_t s = h->stream;
        std::vector<double> sc(SC_COUNT);
        HIPCHK(hipMemcpyAsync(sc.data(), h->sc, SC_COUNT * sizeof(double), hipMemcpyDeviceToHost, s));
        if (y) HIPCHK(hipMemcpyAsync(y, h->y, h->m * sizeof(double), hipMemcpyDeviceToHost, s));
        if (V) HIPCHK(hipMemcpyAsync(V, h->V, (size_t)h->n * 16 * sizeof(double), hipMemcpyDeviceToHost, s));
        if (zbar) HIPCHK(hipMemcpyAsync(zbar, h->zbar, h->m * sizeof(double), hipMemcpyDeviceToHost, s));
        if (Pbar && h->sketch)
            HIPCHK(hipMemcpyAsync(Pbar, h->P, (size_t)h->n * h->r * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (scal) {
            scal[0] = sc[SC_F];
            scal[1] = sc[SC_TAU];
            scal[2] = sc[SC_CBAR];
            scal[3] = sc[SC_CX];
            scal[4] = sc[SC_GAP];
            scal[5] = sc[SC_INF];
            scal[6] = sc[SC_THETA1];
            scal[7] = sc[SC_NDESC];
        }
        return USBS_OK;
    } catch (const DevError &e) {
        return fail(h, e);
    }
}

int usbs_get_test_matrix(usbs_handle *h, float *psi_out) {
    if (!h || !h->ready) return USBS_E_STATE;
    if (!psi_out || !h->sketch) {
        set_err(h, "usbs_get_test_matrix: no sketch or NULL output");
        return USBS_E_INVALID;
    }
    try {
        HIPCHK(hipMemcpyAsync(psi_out, h->psi, (size_t)h->n * h->r * sizeof(float), hipMemcpyDeviceToHost,
                              h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        return USBS_OK;
    } catch (const DevError &e) {
        return fail(h, e);
    }
}

int usbs_get_dual(usbs_handle *h, double *y_out) {
    if (!h || !h->ready) return USBS_E_STATE;
    if (!y_out) return USBS_E_INVALID;
    try {
        HIPCHK(hipMemcpyAsync(y_out, h->y, (size_t)h->m * sizeof(double), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        // App. E: y = ||C||_F y_s
        for (int q = 0; q < h->m; ++q) y_out[q] *= h->sigma;
        return USBS_OK;
    } catch (const DevError &e) {
        return fail(h, e);
    }
}

int usbs_get_primal(usbs_handle *h, double *ax_out, double *cx_out, double *V_out, double *S_out, double *eta_out,
                    double *g_out) {
    if (!h || !h->ready) return USBS_E_STATE;
    if (h->primal_at < 0 || h->primal_at != h->iters) {
        set_err(h, "usbs_get_primal: no iteration has run on the current problem");
        return USBS_E_STATE;
    }
    try {
        hipStream_t s = h->stream;
        const int n = h->n, m = h->m, k = h->k;
        std::vector<double> sc(SC_COUNT), st((size_t)k * k);
        HIPCHK(hipMemcpyAsync(sc.data(), h->sc, SC_COUNT * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(st.data(), h->ipm, (size_t)k * k * sizeof(double), hipMemcpyDeviceToHost, s));
        if (ax_out) HIPCHK(hipMemcpyAsync(ax_out, h->AX, (size_t)m * sizeof(double), hipMemcpyDeviceToHost, s));
        std::vector<double> vt;
        if (V_out) {
            vt.resize((size_t)n * 16);
            HIPCHK(hipMemcpyAsync(vt.data(), h->Vn, (size_t)n * 16 * sizeof(double), hipMemcpyDeviceToHost, s));
        }
        HIPCHK(hipStreamSynchronize(s));
        if (V_out)
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < k; ++j) V_out[(size_t)i * k + j] = vt[(size_t)i * 16 + j];
        if (S_out) std::copy(st.begin(), st.end(), S_out);
        if (cx_out) *cx_out = sc[SC_CX];
        if (eta_out) *eta_out = sc[SC_ETA];
        if (g_out) *g_out = sc[SC_G];
        return USBS_OK;
    } catch (const DevError &e) {
        return fail(h, e);
    }
}

int usbs_warm_start(usbs_handle *h, const usbs_problem *grown) { return usbs_pack::warm_prepare(h, grown, true); }

}  // extern "C"

namespace usbs_pack {
// usbs_warm_start; with eval_f = false the closing eigen-solve for f(y0) is left to the
// packed kernel (PACK_INIT_WARM)
int warm_prepare(usbs_handle *h, const usbs_problem *grown, bool eval_f) {
    if (!h || !h->ready) {
        set_err(h, "usbs_warm_start: handle not ready");
        return USBS_E_STATE;
    }
    try {
        TuneScope tsc(h);
        hipStream_t s = h->stream;
        const int n0 = h->n, m0 = h->m, r = h->r, k = h->k;
        HostProblem hp = copy_problem(grown, r);
        if (hp.n < n0 || hp.m < m0)
            throw DevError(USBS_E_INVALID, "usbs_warm_start: the grown problem must keep all vertices and rows");
        if (r == 0 ? !hp.psi.empty() : (hp.psi.empty() && !h->prm.psi_from_seed))
            throw DevError(USBS_E_INVALID, "usbs_warm_start: sketch presence must not change");
        // ---- state of the old problem (scaled units) ----
        const double sig0 = h->sigma, tr0 = h->trace;
        std::vector<double> y0(m0), V0((size_t)n0 * 16), R0((size_t)n0 * 16), U0, lam0;
        HIPCHK(hipMemcpyAsync(y0.data(), h->y, m0 * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(V0.data(), h->V, (size_t)n0 * 16 * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(R0.data(), h->Uritz, (size_t)n0 * 16 * sizeof(double), hipMemcpyDeviceToHost, s));
        if (r > 0) {
            // Nystrom reconstruction of Xbar (App. C.1): Xhat = U diag(lam) U^T
            interleave(s, n0, r, h->P, h->psi, h->W2);
            tn_reduce(s, h->rs, n0, h->W2, 2 * r, 2 * r, h->W2, 2 * r, 2 * r, h->small, 2 * r, 1.0, 0.0);
            nystrom_core(s, n0, r, h->small, h->small + 1024, h->small + 2048, h->flag);
            nn_update(s, n0, h->W2, 2 * r, 2 * r, h->small + 1024, r, r, h->Zp, 16, 1.0, 0.0);
            U0.resize((size_t)n0 * 16);
            lam0.resize(r);
            HIPCHK(hipMemcpyAsync(U0.data(), h->Zp, (size_t)n0 * 16 * sizeof(double), hipMemcpyDeviceToHost, s));
            HIPCHK(hipMemcpyAsync(lam0.data(), h->small + 2048, r * sizeof(double), hipMemcpyDeviceToHost, s));
        }
        HIPCHK(hipStreamSynchronize(s));
        // ---- the grown problem ----
        free_problem(h);
        h->ready = false;
        h->primal_at = -1;
        h->hp = std::move(hp);
        set_geometry(h, h->hp.n);
        upload(h);
        autotune(h);
        set_tuning(&h->tune);
        const int n = h->n, m = h->m;
        init_scalars(h);
        // y: pad with zeros; y_s = y / ||C||_F rescales by sigma_old / sigma_new
        std::vector<double> y(m, 0.0);
        for (int q = 0; q < m0; ++q) y[q] = y0[q] * sig0 / h->sigma;
        HIPCHK(hipMemcpyAsync(h->y, y.data(), m * sizeof(double), hipMemcpyHostToDevice, s));
        // V and the Ritz block: zero rows for the new vertices, re-orthonormalised
        std::vector<double> Vp((size_t)n * 16, 0.0), Rp((size_t)n * 16, 0.0);
        std::copy(V0.begin(), V0.end(), Vp.begin());
        std::copy(R0.begin(), R0.end(), Rp.begin());
        HIPCHK(hipMemcpyAsync(h->Zp, Vp.data(), (size_t)n * 16 * sizeof(double), hipMemcpyHostToDevice, s));
        set_int(s, h->zdead, 16, 0);
        cholqr2(h, h->Zp, 16, k, h->W2, 16, h->V, 16, h->zdead);
        HIPCHK(hipMemcpyAsync(h->Ubuf, Rp.data(), (size_t)n * 16 * sizeof(double), hipMemcpyHostToDevice, s));
        set_int(s, h->flag, 16, 0);
        cholqr2(h, h->Ubuf, 16, 16, h->W2, 16, h->Uritz, 16, h->flag);
        // Xbar0 = padded Xhat in the new scaling (X_s = X / trace)
        double tau = 0.0, cbar = 0.0;
        if (r > 0) {
            std::vector<double> Up((size_t)n * 16, 0.0), K(r * r, 0.0);
            std::copy(U0.begin(), U0.end(), Up.begin());
            for (int j = 0; j < r; ++j) {
                const double lj = lam0[j] * tr0 / h->trace;
                K[j * r + j] = lj;
                tau += lj;
            }
            HIPCHK(hipMemcpyAsync(h->Zp, Up.data(), (size_t)n * 16 * sizeof(double), hipMemcpyHostToDevice, s));
            HIPCHK(hipMemcpyAsync(h->Kc, K.data(), r * r * sizeof(double), hipMemcpyHostToDevice, s));
            // <C_s, Xhat> = sum_j lam_j u_j^T C_s u_j
            apply_C(h, h->Zp, 16, h->CV, 16, r);
            tn_reduce(s, h->rs, n, h->Zp, 16, r, h->CV, 16, r, h->TUU, r, 1.0, 0.0);
            std::vector<double> uc(r * r);
            HIPCHK(hipMemcpyAsync(uc.data(), h->TUU, r * r * sizeof(double), hipMemcpyDeviceToHost, s));
            // zbar = A(Xhat); P = Xhat Psi = U (K (U^T Psi))
            lowrank_A(s, m, h->kptr, h->ti, h->tj, h->tv, h->Zp, 16, r, h->Kc, 1.0, nullptr, nullptr, 0.0, h->zbar,
                      0.0);
            tn_reduce_f(s, h->rs, n, h->Zp, 16, r, h->psi, r, r, h->VtPsi, r, 1.0);
            HIPCHK(hipStreamSynchronize(s));
            for (int j = 0; j < r; ++j) cbar += K[j * r + j] * uc[j * r + j];
            std::vector<double> Ut(r * r);
            HIPCHK(hipMemcpyAsync(Ut.data(), h->VtPsi, r * r * sizeof(double), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            for (int j = 0; j < r; ++j)
                for (int c = 0; c < r; ++c) Ut[j * r + c] *= K[j * r + j];
            HIPCHK(hipMemcpyAsync(h->Hsk, Ut.data(), r * r * sizeof(double), hipMemcpyHostToDevice, s));
            nn_update(s, n, h->Zp, 16, r, h->Hsk, r, r, h->P, r, 1.0, 0.0);
        } else {
            fill(s, m, 0.0, h->zbar);
        }
        const double tc[2] = {tau, cbar};
        HIPCHK(hipMemcpyAsync(h->sc + SC_TAU, tc, 2 * sizeof(double), hipMemcpyHostToDevice, s));
        if (eval_f) {
            // f(y0) with a tight tolerance
            shift_operator(h, h->y);
            lanczos(h, h->Uritz, k, h->prm.lanczos_tol_final, std::sqrt(h->prm.lanczos_tol_final),
                    std::max(h->prm.lanczos_max_restarts, 30), false, kCertifyMinCycles);
            recompute_f(s, h->theta, h->y, h->b, m, h->rs, h->sc, 0);
        }
        HIPCHK(hipStreamSynchronize(s));
        h->ready = true;
        return USBS_OK;
    } catch (const DevError &e) {
        return fail(h, e);
    }
}

}  // namespace usbs_pack

// ===========================================================================
// packed solver: host side
// ===========================================================================
namespace {

void fill_desc(const usbs_handle *h, PackDesc &d) {
    std::memset(&d, 0, sizeof(d));
    const usbs_params &p = h->prm;
    d.n = h->n;
    d.m = h->m;
    d.k = h->k;
    d.kc = h->kc;
    d.kp = h->kp;
    d.r = h->r;
    d.steps = h->steps;
    d.ldb = h->ldb;
    d.prec = h->prec;
    d.n_iso = h->n_iso;
    d.n_offt = h->has_offc ? h->n_offt : 0;
    d.has_ineq = h->has_ineq ? 1 : 0;
    d.sketch = h->sketch ? 1 : 0;
    d.max_restarts = p.lanczos_max_restarts;
    d.max_iters = p.max_iters;
    d.val_scale = h->val_scale;
    d.tol = p.lanczos_tol;
    d.tol_rest = p.lanczos_tol_rest > 0.0 ? p.lanczos_tol_rest : std::sqrt(p.lanczos_tol);
    d.tol_final = p.lanczos_tol_final;
    d.alpha = p.alpha;
    d.rho = p.rho;
    d.eps_gap = p.eps_gap;
    d.eps_inf = p.eps_infeas;
    d.seed = p.seed;
    d.rowptr = h->rowptr;
    d.col = h->col;
    d.val_cur = h->val_cur;
    d.val_c = h->val_c;
    d.cbase = h->cbase;
    d.cdiag = h->cdiag;
    d.dshift = h->dshift;
    d.dptr = h->dptr;
    d.dk = h->dk;
    d.dv = h->dv;
    d.off_slot = h->off_slot;
    d.off_ptr = h->off_ptr;
    d.off_k = h->off_k;
    d.off_hv = h->off_hv;
    d.kptr = h->kptr;
    d.ti = h->ti;
    d.tj = h->tj;
    d.tv = h->tv;
    d.b = h->b;
    d.ineq = h->ineq;
    d.psi = h->psi;
    d.y = h->y;
    d.yc = h->yc;
    d.nu = h->nu;
    d.dnu = h->dnu;
    d.zbar = h->zbar;
    d.AX = h->AX;
    d.evec = h->evec;
    d.V = h->V;
    d.Vn = h->Vn;
    d.CV = h->CV;
    d.Uritz = h->Uritz;
    d.P = h->P;
    d.Ucpl = h->Ucpl;
    d.iso_idx = h->iso_idx;
    d.plan = h->plan;
    d.Bm = h->Bm;
    d.W = h->W;
    d.Wt = h->Wt;
    d.W2 = h->W2;
    d.Ubuf = h->Ubuf;
    d.Zp = h->Zp;
    d.Tm = h->Tm;
    d.theta = h->theta;
    d.Ysm = h->Ysm;
    d.TUU = h->TUU;
    d.RtR = h->RtR;
    d.Zc = h->Zc;
    d.Hred = h->Hred;
    d.Hg = h->Hg;
    d.coef = h->coef;
    d.Rsv = h->Rsv;
    d.Rinv = h->Rinv;
    d.res = h->res;
    d.Hd = h->Hd;
    d.dead = h->dead;
    d.flag = h->flag;
    d.zdead = h->zdead;
    d.raw = h->raw;
    d.qp = h->qp;
    d.ipm = h->ipm;
    d.VCV = h->VCV;
    d.Gy = h->Gy;
    d.Kc = h->Kc;
    d.Qp = h->Qp;
    d.Hsk = h->Hsk;
    d.VtPsi = h->VtPsi;
    d.hz = h->hz;
    d.sc = h->sc;
}

}  // namespace

namespace usbs_pack {

namespace {
void drop_graph(Runner &R) {
    if (R.graph_exec) (void)hipGraphExecDestroy(R.graph_exec);
    if (R.graph) (void)hipGraphDestroy(R.graph);
    R.graph_exec = nullptr;
    R.graph = nullptr;
    R.graph_count = R.graph_iters = 0;
}
// the steps of one launch over the first na table entries
void issue_launch(Runner &R, int na, int iters) {
    HIPCHK(hipMemcpyAsync(R.desc_dev, R.desc_host, na * sizeof(PackDesc), hipMemcpyHostToDevice, R.stream));
    HIPCHK(hipMemcpyAsync(R.state_dev, R.state_host, na * sizeof(PackState), hipMemcpyHostToDevice, R.stream));
    packed_launch(R.stream, R.desc_dev, R.state_dev, na, iters);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(R.state_host, R.state_dev, na * sizeof(PackState), hipMemcpyDeviceToHost, R.stream));
}
// capture the launch steps as a graph (the host tables are read when the graph runs)
bool capture_launch(Runner &R, int na, int iters) {
    drop_graph(R);
    if (hipStreamBeginCapture(R.stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return false;
    bool ok = true;
    try {
        issue_launch(R, na, iters);
    } catch (const DevError &) {
        ok = false;
    }
    hipGraph_t g = nullptr;
    if (hipStreamEndCapture(R.stream, &g) != hipSuccess || !ok || !g) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        return false;
    }
    hipGraphExec_t ge = nullptr;
    if (hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        return false;
    }
    R.graph = g;
    R.graph_exec = ge;
    R.graph_count = na;
    R.graph_iters = iters;
    return true;
}
}  // namespace

Runner::~Runner() {
    drop_graph(*this);
    if (desc_dev) (void)hipFreeAsync(desc_dev, stream);
    if (state_dev) (void)hipFreeAsync(state_dev, stream);
    (void)hipStreamSynchronize(stream);
    if (desc_host) (void)hipHostFree(desc_host);
    if (state_host) (void)hipHostFree(state_host);
}

PackState begin(const usbs_handle *h, int init) {
    PackState s;
    std::memset(&s, 0, sizeof(s));
    s.iters = h->iters;
    s.null_run = h->null_run;
    s.lz_unconverged = h->lz_unconverged;
    s.recoveries = h->recoveries;
    s.matvecs = h->matvecs;
    s.init = init;
    s.done = PACK_RUNNING;
    return s;
}

int launch(Runner &R, usbs_handle *const *hs, PackState *st, int count, int iters, std::string *err) {
    try {
        std::vector<int> act;
        for (int q = 0; q < count; ++q)
            if (st[q].done == PACK_RUNNING) act.push_back(q);
        const int na = (int)act.size();
        if (na == 0) return USBS_OK;
        if (na > R.cap) {
            drop_graph(R);   // the graph holds the old table addresses
            if (R.desc_dev) HIPCHK(hipFreeAsync(R.desc_dev, R.stream));
            if (R.state_dev) HIPCHK(hipFreeAsync(R.state_dev, R.stream));
            HIPCHK(hipStreamSynchronize(R.stream));
            if (R.desc_host) HIPCHK(hipHostFree(R.desc_host));
            if (R.state_host) HIPCHK(hipHostFree(R.state_host));
            R.desc_dev = nullptr;
            R.state_dev = nullptr;
            R.desc_host = nullptr;
            R.state_host = nullptr;
            R.cap = 0;
            const int cap = std::max(na, 64);
            HIPCHK(hipMallocAsync((void **)&R.desc_dev, cap * sizeof(PackDesc), R.stream));
            HIPCHK(hipMallocAsync((void **)&R.state_dev, cap * sizeof(PackState), R.stream));
            HIPCHK(hipHostMalloc((void **)&R.desc_host, cap * sizeof(PackDesc), hipHostMallocDefault));
            HIPCHK(hipHostMalloc((void **)&R.state_host, cap * sizeof(PackState), hipHostMallocDefault));
            R.cap = cap;
        }
        for (int a = 0; a < na; ++a) {
            const int q = act[a];
            usbs_handle *h = hs[q];
            if (!h || !h->ready) throw DevError(USBS_E_STATE, "packed launch: handle not ready");
            if (h->n < 2 * (16 + 8)) throw DevError(USBS_E_INVALID, "packed launch: n < 48");
            fill_desc(h, R.desc_host[a]);
            R.state_host[a] = st[q];
        }
        bool replayed = false;
        if (R.stream && !R.graph_failed) {
            if (!(R.graph_exec && R.graph_count == na && R.graph_iters == iters) && !capture_launch(R, na, iters))
                R.graph_failed = true;
            if (R.graph_exec && R.graph_count == na && R.graph_iters == iters) {
                HIPCHK(hipGraphLaunch(R.graph_exec, R.stream));
                R.graph_replays++;
                replayed = true;
            }
        }
        if (!replayed) issue_launch(R, na, iters);
        HIPCHK(hipStreamSynchronize(R.stream));
        for (int a = 0; a < na; ++a) {
            const int q = act[a];
            usbs_handle *h = hs[q];
            st[q] = R.state_host[a];
            if (st[q].swapped) std::swap(h->V, h->Vn);
            st[q].swapped = 0;
            if (st[q].iters != h->iters) h->primal_at = st[q].iters;
            h->iters = st[q].iters;
            h->null_run = st[q].null_run;
            h->lz_unconverged = st[q].lz_unconverged;
            h->recoveries = st[q].recoveries;
            h->matvecs = st[q].matvecs;
            for (int ph = 0; ph < kPackPhases; ++ph) h->pack_ticks[ph] += st[q].ticks[ph];
            std::memset(st[q].ticks, 0, sizeof(st[q].ticks));
        }
        return USBS_OK;
    } catch (const DevError &e) {
        if (err) *err = e.what();
        return e.code;
    }
}

int finish(usbs_handle *h, const PackState &st, usbs_result *res, double secs) {
    try {
        if (st.done == PACK_FAILED) throw DevError(USBS_E_NUMERIC, "non-finite iterate or failed interior point solve");
        const int status = st.done == PACK_CONVERGED ? USBS_OK : USBS_NOT_CONVERGED;
        fill_result(h, res, nullptr, nullptr, nullptr, status, st.solve_iters, secs);
        return status;
    } catch (const DevError &e) {
        return fail(h, e);
    }
}

}  // namespace usbs_pack

extern "C" {

int usbs_solve_packed(usbs_handle *const *hs, int32_t count, int32_t iters_per_launch, void *stream,
                      usbs_result *res, int32_t *status) {
    if (!hs || count < 1 || iters_per_launch < 1) return USBS_E_INVALID;
    int dev = -1;
    for (int q = 0; q < count; ++q) {
        if (!hs[q] || !hs[q]->ready) return USBS_E_STATE;
        if (dev < 0) dev = hs[q]->dev;
        if (hs[q]->dev != dev) {
            set_err(hs[q], "usbs_solve_packed: handles of different devices");
            return USBS_E_INVALID;
        }
        for (int p = 0; p < q; ++p)
            if (hs[p] == hs[q]) {
                set_err(hs[q], "usbs_solve_packed: a handle is listed twice");
                return USBS_E_INVALID;
            }
    }
    try {
        for (int q = 0; q < count; ++q) HIPCHK(hipStreamSynchronize(hs[q]->stream));
    } catch (const DevError &e) {
        return fail(hs[0], e);
    }
    usbs_pack::Runner R((hipStream_t)stream);
    std::vector<PackState> st(count);
    std::vector<double> secs(count, 0.0);
    for (int q = 0; q < count; ++q) st[q] = usbs_pack::begin(hs[q], PACK_INIT_NONE);
    const auto t0 = std::chrono::steady_clock::now();
    int rc = USBS_OK;
    for (;;) {
        bool any = false;
        for (int q = 0; q < count; ++q) any |= st[q].done == PACK_RUNNING;
        if (!any) break;
        std::string err;
        rc = usbs_pack::launch(R, hs, st.data(), count, iters_per_launch, &err);
        if (rc < 0) {
            for (int q = 0; q < count; ++q) set_err(hs[q], err);
            return rc;
        }
        const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        for (int q = 0; q < count; ++q) {
            if (st[q].done != PACK_RUNNING) {
                if (secs[q] == 0.0) secs[q] = el;
            } else if (hs[q]->prm.time_limit > 0.0 && el > hs[q]->prm.time_limit) {
                st[q].stop = 1;   // the next launch certifies f at the centre and stops
            }
        }
    }
    int worst = USBS_OK;
    for (int q = 0; q < count; ++q) {
        const int s = usbs_pack::finish(hs[q], st[q], res ? res + q : nullptr, secs[q]);
        if (status) status[q] = s;
        if (s < 0 && worst >= 0) worst = s;
        else if (s == USBS_NOT_CONVERGED && worst == USBS_OK) worst = s;
    }
    return worst;
}

int usbs_packed_profile(usbs_handle *h, int32_t reset, double *ms_out) {
    if (!h || !h->ready) return USBS_E_STATE;
    try {
        int khz = 0;
        HIPCHK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, h->dev));
        if (khz <= 0) throw DevError(USBS_E_DEVICE, "no device wall-clock rate");
        if (ms_out)
            for (int ph = 0; ph < kPackPhases; ++ph) ms_out[ph] = (double)h->pack_ticks[ph] / (double)khz;
        if (reset) std::memset(h->pack_ticks, 0, sizeof(h->pack_ticks));
        return USBS_OK;
    } catch (const DevError &e) {
        return fail(h, e);
    }
}

}  // extern "C"
