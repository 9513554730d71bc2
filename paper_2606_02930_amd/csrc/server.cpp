// Serving loop: many independent imaginary-time evolutions (one per request)
// advanced concurrently on one device with continuous batching.
//
// Each worker is a host thread with its own context on its own non-blocking
// stream; a request, once admitted, stays on the worker that admitted it and
// that worker advances all its active requests by one time step at a time as
// one batch (ite_step_batch: their local solves share grouped launches and a
// captured graph; each result is bitwise that of the request run alone).  The
// FIFO queue admits the oldest request as soon as the summed footprint of the
// active requests leaves room for it and a worker has a free slot, so short
// requests that arrive while long ones run start at once instead of behind
// them.  Device memory comes from a pool that never returns memory to HIP
// while the server runs: freeing device memory can wait for the whole device,
// which would stall every other worker.
#include "engine.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

using namespace ite;

namespace {

// Size-class pool of device memory shared by the worker contexts.
struct Pool {
    int device = 0;
    std::mutex m;
    std::multimap<size_t, void*> free_;
    std::unordered_map<void*, size_t> size_;
    size_t reserved = 0;

    static size_t round_up(size_t b) {
        if (b <= (size_t(1) << 20)) return (b + 255) & ~size_t(255);
        size_t p = 1;
        while (p < b) p <<= 1;
        const size_t step = p / 16;
        return (b + step - 1) / step * step;
    }
    void* alloc(size_t b) {
        b = round_up(std::max<size_t>(b, 256));
        {
            std::lock_guard<std::mutex> lk(m);
            auto it = free_.lower_bound(b);
            if (it != free_.end() && it->first <= b + b / 4) {
                void* p = it->second;
                free_.erase(it);
                return p;
            }
        }
        void* p = nullptr;
        if (hipSetDevice(device) != hipSuccess || hipMalloc(&p, b) != hipSuccess) return nullptr;
        std::lock_guard<std::mutex> lk(m);
        size_[p] = b;
        reserved += b;
        return p;
    }
    void release(void* p) {
        if (!p) return;
        std::lock_guard<std::mutex> lk(m);
        auto it = size_.find(p);
        if (it != size_.end()) free_.emplace(it->second, p);
    }
    ~Pool() {
        (void)hipSetDevice(device);
        for (auto& kv : size_) (void)hipFree(kv.first);
    }
    static void* cb_alloc(size_t b, void* user) { return static_cast<Pool*>(user)->alloc(b); }
    static void cb_free(void* p, void* user) { static_cast<Pool*>(user)->release(p); }
};

std::vector<int> full_bonds(int L, const std::vector<int>& d, int chi) {
    std::vector<double> left(L + 1, 1.0), right(L + 1, 1.0);
    for (int i = 0; i < L; ++i) left[i + 1] = std::min(1e18, left[i] * d[i]);
    for (int i = L - 1; i >= 0; --i) right[i] = std::min(1e18, right[i + 1] * d[i]);
    std::vector<int> D(L + 1);
    for (int i = 0; i <= L; ++i) D[i] = (int)std::min<double>({(double)chi, left[i], right[i]});
    return D;
}

struct Req {
    long long id = 0;
    int L = 0;
    std::vector<int> d, w;
    std::vector<std::vector<double>> W, sp;
    int chi_max = 1, pad_full = 0;
    std::vector<double> grid;
    ite_step_opts o{};
    double fp = 0.0;
    // state (guarded by the server mutex unless noted)
    int status = ITE_REQ_PENDING, error = 0, worker = -1, k = 0;
    double tau = 0.0, energy = 0.0, t_submit = 0.0, t_admit = 0.0, t_done = 0.0;
    std::string err;
    std::vector<ite_step_report> reps;
    std::vector<int> chi;
    std::vector<std::vector<double>> A;
    // device handles: touched only by the owning worker
    ite_mpo* H = nullptr;
    ite_mps* psi = nullptr;
};

}  // namespace

struct ite_server {
    ite_server_opts o{};
    Pool pool;
    std::vector<ite_ctx*> ctx;
    std::vector<hipStream_t> streams;
    std::vector<std::thread> threads;
    std::mutex m;
    std::condition_variable cv_work, cv_done;
    std::unordered_map<long long, std::shared_ptr<Req>> reqs;
    std::deque<std::shared_ptr<Req>> pending;
    std::vector<std::vector<std::shared_ptr<Req>>> active;
    std::vector<size_t> rr;
    double active_bytes = 0.0;
    long long next_id = 1;
    bool stop = false;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    void worker(int wi);
    void finish(const std::shared_ptr<Req>& r, int wi, int status, int code, const std::string& msg);
};

void ite_server::finish(const std::shared_ptr<Req>& r, int wi, int status, int code, const std::string& msg) {
    ite_ctx* c = ctx[wi];
    if (r->psi) ite_mps_destroy(r->psi);
    if (r->H) ite_mpo_destroy(r->H);
    r->psi = nullptr;
    r->H = nullptr;
    (void)c;
    std::lock_guard<std::mutex> lk(m);
    r->status = status;
    r->error = code;
    r->err = msg;
    r->t_done = now();
    active_bytes -= r->fp;
    auto& a = active[wi];
    a.erase(std::remove(a.begin(), a.end(), r), a.end());
    cv_done.notify_all();
    cv_work.notify_all();
}

void ite_server::worker(int wi) {
    ite_ctx* c = ctx[wi];
    // this thread's allocations and copies (admissions) may overlap another
    // worker's graph capture: they do not touch its stream
    hipStreamCaptureMode relaxed = hipStreamCaptureModeRelaxed;
    (void)hipThreadExchangeStreamCaptureMode(&relaxed);
    for (;;) {
        std::shared_ptr<Req> r;
        std::vector<std::shared_ptr<Req>> batch;
        {
            std::unique_lock<std::mutex> lk(m);
            for (;;) {
                if (stop) return;
                if (!pending.empty() && (int)active[wi].size() < o.max_active &&
                    active_bytes + pending.front()->fp <= o.mem_cap) {
                    r = pending.front();
                    pending.pop_front();
                    r->status = ITE_REQ_ACTIVE;
                    r->worker = wi;
                    r->t_admit = now();
                    active_bytes += r->fp;
                    active[wi].push_back(r);
                    break;
                }
                if (!active[wi].empty()) {
                    batch = active[wi];
                    break;
                }
                cv_work.wait(lk);
            }
        }
        if (r) {
            // a fresh admission: its tensors, then back to admit more before
            // the next batched step
            std::vector<const double*> Wp(r->L), Sp(r->L);
            for (int i = 0; i < r->L; ++i) {
                Wp[i] = r->W[i].data();
                Sp[i] = r->sp[i].data();
            }
            int rc = ite_mpo_load(c, r->L, r->d.data(), r->w.data(), Wp.data(), &r->H);
            if (rc == ITE_OK)
                rc = ite_mps_create(c, r->L, r->d.data(), Sp.data(), r->chi_max, r->pad_full, &r->psi);
            if (rc != ITE_OK) finish(r, wi, ITE_REQ_FAILED, rc, ite_last_error(c));
            continue;
        }
        // one time step of every active request of this worker, as one batch:
        // request j goes from grid[k] to grid[k + 1]
        const int n = (int)batch.size();
        std::vector<ite_mps*> P(n);
        std::vector<const ite_mpo*> Hs(n);
        std::vector<double> hs(n);
        std::vector<const ite_step_opts*> Os(n);
        for (int j = 0; j < n; ++j) {
            Req& q = *batch[j];
            const double dtau = q.grid[q.k + 1] - q.grid[q.k];
            P[j] = q.psi;
            Hs[j] = q.H;
            hs[j] = q.o.scheme == ITE_SCHEME_TRAP ? 0.5 * dtau : dtau;
            Os[j] = &q.o;
        }
        std::vector<ite_step_report> reps(n);
        std::vector<int> st(n, ITE_OK);
        const int brc = ite_step_batch(c, n, P.data(), Hs.data(), hs.data(), Os.data(), reps.data(), st.data());
        const std::string bmsg = ite_last_error(c);
        for (int j = 0; j < n; ++j) {
            const std::shared_ptr<Req>& q = batch[j];
            int rc = brc != ITE_OK && st[j] == ITE_OK && brc != ITE_ENONFINITE ? brc : st[j];
            if (rc != ITE_OK) {
                finish(q, wi, ITE_REQ_FAILED, rc, bmsg);
                continue;
            }
            ite_step_report rep = reps[j];
            ite_mps_set_tau(q->psi, q->grid[q->k + 1]);
            rep.tau = q->grid[q->k + 1];
            bool last;
            {
                std::lock_guard<std::mutex> lk(m);
                q->reps.push_back(rep);
                q->k += 1;
                q->tau = rep.tau;
                q->energy = rep.energy;
                last = q->k + 1 >= (int)q->grid.size();
            }
            if (!last) continue;
            std::vector<int> chi(q->L + 1);
            rc = ite_mps_export(q->psi, chi.data(), nullptr);
            std::vector<std::vector<double>> A(q->L);
            std::vector<double*> Ap(q->L);
            if (rc == ITE_OK) {
                for (int i = 0; i < q->L; ++i) {
                    A[i].resize((size_t)chi[i] * q->d[i] * chi[i + 1]);
                    Ap[i] = A[i].data();
                }
                rc = ite_mps_export(q->psi, chi.data(), Ap.data());
            }
            if (rc != ITE_OK) {
                finish(q, wi, ITE_REQ_FAILED, rc, ite_last_error(c));
                continue;
            }
            q->chi = std::move(chi);
            q->A = std::move(A);
            finish(q, wi, ITE_REQ_DONE, ITE_OK, "");
        }
    }
}

namespace {

void fill_info(const Req& r, ite_request_info* info) {
    info->status = r.status;
    info->error = r.error;
    info->worker = r.worker;
    info->n_steps = r.k;
    info->n_grid = (int)r.grid.size() - 1;
    info->tau = r.tau;
    info->energy = r.energy;
    info->footprint = r.fp;
    info->t_submit = r.t_submit;
    info->t_admit = r.t_admit;
    info->t_done = r.t_done;
}

}  // namespace

extern "C" {

double ite_request_footprint(int L, const int* d, const int* w, int chi_max, int krylov_dim) {
    if (L < 2 || !d || !w || chi_max < 1 || krylov_dim < 1) return -1.0;
    std::vector<int> dv(d, d + L);
    const std::vector<int> D = full_bonds(L, dv, chi_max);
    double mps = 0.0, envs = 0.0, nmax = 0.0, xmax = 0.0, zmax = 0.0;
    for (int i = 0; i < L; ++i) mps += (double)D[i] * d[i] * D[i + 1];
    for (int i = 0; i <= L; ++i) envs += (2.0 * w[i] + 1.0) * D[i] * D[i];
    for (int i = 0; i + 1 < L; ++i) {
        const double n = (double)D[i] * d[i] * d[i + 1] * D[i + 2];
        nmax = std::max(nmax, n);
        const double I = (double)std::max(w[i], w[i + 2]) * d[i] * d[i + 1];
        xmax = std::max(xmax, (double)D[i] * I * D[i + 2]);
        const double p = std::min((double)D[i] * d[i], (double)d[i + 1] * D[i + 2]);
        zmax = std::max(zmax, p * ((double)D[i] * d[i] + (double)d[i + 1] * D[i + 2]));
    }
    // psi and its working copy, three environment kinds, Krylov basis and
    // solve vectors, the two contraction intermediates, the split work matrix,
    // its Gram partials and the second buffer of its data columns,
    // low-precision shadows (at most half of FP64)
    const double doubles = 2.0 * mps + envs + (krylov_dim + 8.0) * nmax + 2.0 * xmax + 3.0 * zmax +
                           0.5 * (envs + xmax + nmax);
    return 8.0 * doubles + (double)(64 << 20);
}

int ite_server_create(const ite_server_opts* o, ite_server** out) {
    if (!o || !out) return ITE_EINVAL;
    *out = nullptr;
    if (o->workers < 1 || o->workers > 64 || o->max_active < 1 || !(o->mem_cap > 0.0)) return ITE_EINVAL;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || o->device < 0 || o->device >= n) return ITE_EDEVICE;
    std::unique_ptr<ite_server> s(new ite_server);
    s->o = *o;
    s->pool.device = o->device;
    if (hipSetDevice(o->device) != hipSuccess) return ITE_EDEVICE;
    ite_allocator al{Pool::cb_alloc, Pool::cb_free, &s->pool};
    for (int i = 0; i < o->workers; ++i) {
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            ite_server_destroy(s.release());
            return ITE_EDEVICE;
        }
        s->streams.push_back(st);
        ite_ctx* c = nullptr;
        const int rc = ite_ctx_create(o->device, st, &al, &c);
        if (rc != ITE_OK) {
            ite_server_destroy(s.release());
            return rc;
        }
        s->ctx.push_back(c);
    }
    s->active.resize(o->workers);
    s->rr.assign(o->workers, 0);
    for (int i = 0; i < o->workers; ++i) s->threads.emplace_back([srv = s.get(), i] { srv->worker(i); });
    *out = s.release();
    return ITE_OK;
}

int ite_server_destroy(ite_server* s) {
    if (!s) return ITE_EINVAL;
    {
        std::lock_guard<std::mutex> lk(s->m);
        s->stop = true;
    }
    s->cv_work.notify_all();
    for (auto& t : s->threads) t.join();
    // requests still on a worker: free their handles from this thread (the
    // workers have stopped)
    for (size_t wi = 0; wi < s->active.size(); ++wi)
        for (auto& r : s->active[wi]) {
            if (r->psi) ite_mps_destroy(r->psi);
            if (r->H) ite_mpo_destroy(r->H);
            r->psi = nullptr;
            r->H = nullptr;
        }
    for (ite_ctx* c : s->ctx) ite_ctx_destroy(c);
    for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
    delete s;
    return ITE_OK;
}

int ite_server_submit(ite_server* s, const ite_request* q, long long* id) {
    if (!s || !q || !id) return ITE_EINVAL;
    *id = 0;
    try {
        auto r = std::make_shared<Req>();
        if (q->L < 2 || !q->d || !q->w || !q->W || !q->spinors || q->chi_max < 1) return ITE_EINVAL;
        r->L = q->L;
        r->d.assign(q->d, q->d + q->L);
        r->w.assign(q->w, q->w + q->L + 1);
        if (r->w[0] != 1 || r->w[q->L] != 1) return ITE_EINVAL;
        for (int i = 0; i < q->L; ++i) {
            if (r->d[i] < 1 || r->d[i] > 8 || r->w[i] < 1 || r->w[i] > 16 || !q->W[i] || !q->spinors[i])
                return ITE_EINVAL;
            const size_t nw = (size_t)r->w[i] * r->w[i + 1] * r->d[i] * r->d[i];
            r->W.emplace_back(q->W[i], q->W[i] + nw);
            r->sp.emplace_back(q->spinors[i], q->spinors[i] + r->d[i]);
        }
        r->chi_max = q->chi_max;
        r->pad_full = q->pad_full;
        r->o = q->opts;
        int n = 0;
        if (ite_loggrid(q->tau0, q->tau1, q->ratio, nullptr, 0, &n) == ITE_EINVAL && n == 0) return ITE_EINVAL;
        r->grid.resize(n);
        if (ite_loggrid(q->tau0, q->tau1, q->ratio, r->grid.data(), n, &n) != ITE_OK) return ITE_EINVAL;
        r->fp = ite_request_footprint(r->L, r->d.data(), r->w.data(), r->chi_max, std::max(1, r->o.krylov_dim));
        if (r->fp > s->o.mem_cap) return ITE_ENOMEM;
        std::lock_guard<std::mutex> lk(s->m);
        r->id = s->next_id++;
        r->t_submit = s->now();
        s->reqs[r->id] = r;
        s->pending.push_back(r);
        *id = r->id;
    } catch (const std::bad_alloc&) {
        return ITE_ENOMEM;
    }
    s->cv_work.notify_all();
    return ITE_OK;
}

int ite_server_info(ite_server* s, long long id, ite_request_info* info) {
    if (!s || !info) return ITE_EINVAL;
    std::lock_guard<std::mutex> lk(s->m);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return ITE_EINVAL;
    fill_info(*it->second, info);
    return ITE_OK;
}

int ite_server_wait(ite_server* s, long long id, double timeout_s, ite_request_info* info) {
    if (!s || !info) return ITE_EINVAL;
    std::unique_lock<std::mutex> lk(s->m);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return ITE_EINVAL;
    std::shared_ptr<Req> r = it->second;
    auto done = [&] { return r->status == ITE_REQ_DONE || r->status == ITE_REQ_FAILED; };
    if (timeout_s < 0) s->cv_done.wait(lk, done);
    else s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), done);
    fill_info(*r, info);
    return done() ? ITE_OK : ITE_ESTATE;
}

int ite_server_reports(ite_server* s, long long id, ite_step_report* out, int cap, int* n) {
    if (!s || !n) return ITE_EINVAL;
    std::lock_guard<std::mutex> lk(s->m);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return ITE_EINVAL;
    const Req& r = *it->second;
    *n = (int)r.reps.size();
    if (out)
        for (int i = 0; i < std::min(cap, *n); ++i) out[i] = r.reps[i];
    return ITE_OK;
}

int ite_server_state(ite_server* s, long long id, int* chi, double* const* A) {
    if (!s || !chi) return ITE_EINVAL;
    std::lock_guard<std::mutex> lk(s->m);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return ITE_EINVAL;
    const Req& r = *it->second;
    if (r.status != ITE_REQ_DONE) return ITE_ESTATE;
    std::copy(r.chi.begin(), r.chi.end(), chi);
    if (A)
        for (int i = 0; i < r.L; ++i) {
            if (!A[i]) return ITE_EINVAL;
            std::memcpy(A[i], r.A[i].data(), r.A[i].size() * sizeof(double));
        }
    return ITE_OK;
}

int ite_server_release(ite_server* s, long long id) {
    if (!s) return ITE_EINVAL;
    std::lock_guard<std::mutex> lk(s->m);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return ITE_EINVAL;
    if (it->second->status != ITE_REQ_DONE && it->second->status != ITE_REQ_FAILED) return ITE_ESTATE;
    s->reqs.erase(it);
    return ITE_OK;
}

double ite_server_clock(const ite_server* s) { return s ? s->now() : 0.0; }

int ite_server_error(ite_server* s, long long id, char* buf, int cap) {
    if (!s || !buf || cap < 1) return ITE_EINVAL;
    std::lock_guard<std::mutex> lk(s->m);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return ITE_EINVAL;
    const std::string& e = it->second->err;
    const size_t k = std::min<size_t>(e.size(), (size_t)cap - 1);
    std::memcpy(buf, e.data(), k);
    buf[k] = '\0';
    return ITE_OK;
}

}  // extern "C"
