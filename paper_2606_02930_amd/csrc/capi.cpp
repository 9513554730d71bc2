// extern "C" entry points: argument checks, error translation (no C++
// exception crosses the boundary), and the parity-test building blocks.
#include "engine.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>

using namespace ite;

namespace {

template <typename F>
int guarded(ite_ctx* c, F&& f) {
    try {
        if (c) c->err.clear();
        f();
        return ITE_OK;
    } catch (const Error& e) {
        if (c) c->err = e.what();
        return e.code;
    } catch (const std::bad_alloc&) {
        if (c) c->err = "host allocation failed";
        return ITE_ENOMEM;
    } catch (const std::exception& e) {
        if (c) c->err = e.what();
        return ITE_EDEVICE;
    } catch (...) {
        if (c) c->err = "unknown error";
        return ITE_EDEVICE;
    }
}

void set_device(ite_ctx* c) { HIP_CHECK(hipSetDevice(c->device)); }

bool opts_ok(const ite_step_opts* o) { return o != nullptr; }

// A CSR matrix uploaded for one call of a parity-test building block.
struct TmpCsr {
    ite_ctx* c = nullptr;
    char* blk = nullptr;
    CsrDev cs;
    TmpCsr(ite_ctx* ctx, const std::vector<double>& M, int O, int I) : c(ctx) {
        std::vector<int> rowptr(1, 0), col;
        std::vector<double> val;
        for (int o = 0; o < O; ++o) {
            for (int i = 0; i < I; ++i)
                if (M[(size_t)o * I + i] != 0.0) {
                    col.push_back(i);
                    val.push_back(M[(size_t)o * I + i]);
                }
            rowptr.push_back((int)col.size());
        }
        const size_t vb = (val.size() * 8 + 255) & ~size_t(255);
        const size_t rb = (rowptr.size() * 4 + 255) & ~size_t(255);
        const size_t cb = (col.size() * 4 + 255) & ~size_t(255);
        blk = static_cast<char*>(dev_alloc(c, vb + rb + cb + 256));
        cs.I = I;
        cs.O = O;
        cs.nnz = (int)val.size();
        cs.val = reinterpret_cast<double*>(blk);
        cs.rowptr = reinterpret_cast<int*>(blk + vb);
        cs.col = reinterpret_cast<int*>(blk + vb + rb);
        h2d_wait(c, cs.val, val.data(), val.size() * 8);
        h2d_wait(c, cs.rowptr, rowptr.data(), rowptr.size() * 4);
        h2d_wait(c, cs.col, col.data(), col.size() * 4);
    }
    ~TmpCsr() {
        if (blk) {
            (void)hipStreamSynchronize(c->stream);
            dev_free(c, blk);
        }
    }
    TmpCsr(const TmpCsr&) = delete;
    TmpCsr& operator=(const TmpCsr&) = delete;
};

// WW[(p q u), (w s t)] = sum_v W1[w][v][p][s] W2[v][u][q][t]
std::vector<double> pair_matrix(const double* W1h, const double* W2h, int w0, int w1, int w2, int d1, int d2) {
    const int I = w0 * d1 * d2, O = d1 * d2 * w2;
    std::vector<double> M((size_t)O * I, 0.0);
    for (int a = 0; a < w0; ++a)
        for (int s = 0; s < d1; ++s)
            for (int t = 0; t < d2; ++t)
                for (int p = 0; p < d1; ++p)
                    for (int q = 0; q < d2; ++q)
                        for (int u = 0; u < w2; ++u) {
                            double acc = 0.0;
                            for (int v = 0; v < w1; ++v)
                                acc += W1h[(((size_t)a * w1 + v) * d1 + p) * d1 + s] *
                                       W2h[(((size_t)v * w2 + u) * d2 + q) * d2 + t];
                            M[((size_t)(p * d2 + q) * w2 + u) * I + (a * d1 + s) * d2 + t] = acc;
                        }
    return M;
}

}  // namespace

extern "C" {

const char* ite_version(void) { return "ite 0.1 (gfx950)"; }

void ite_default_opts(ite_step_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->scheme = ITE_SCHEME_TRAP;
    o->shift_mode = ITE_SHIFT_TRACK;
    o->shift = 0.0;
    o->chi_max = 200;
    o->cutoff = 1e-10;
    o->tie_rel = 1e-13;
    o->krylov_dim = 10;
    o->max_cycles = 1;
    o->tol_loc = 0.0;
    o->nsweeps = 1;
    o->precision = ITE_PREC_FP64;
    o->max_refine = 0;   // per precision: 1 correction for FP32-IR, 2 for BF16-IR
    o->tol_refine = 0.0;
    o->init_guess = ITE_GUESS_B;
    o->gl_nodes = 2;
    o->rhs_mode = ITE_RHS_PROJECT;
}

int ite_ctx_create(int device, void* hip_stream, const ite_allocator* alloc, ite_ctx** out) {
    if (!out) return ITE_EINVAL;
    *out = nullptr;
    if (alloc && (!alloc->alloc || !alloc->free)) return ITE_EINVAL;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return device < 0 ? ITE_EINVAL : ITE_EDEVICE;
    std::unique_ptr<ite_ctx> c(new ite_ctx);
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    if (alloc) {
        c->alloc = *alloc;
        c->has_alloc = true;
    }
    if (hipSetDevice(device) != hipSuccess) return ITE_EDEVICE;
    // this device's copy of the fixed scratch of ite_mps_sample_noalloc
    const int rc = guarded(c.get(), [&] { noalloc_init(device); });
    if (rc != ITE_OK) return rc;
    *out = c.release();
    return ITE_OK;
}

int ite_ctx_destroy(ite_ctx* c) {
    if (!c) return ITE_EINVAL;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    if (c->side) (void)hipStreamSynchronize(c->side);
    for (auto& g : c->bgraphs) (void)hipGraphExecDestroy(g.exec);
    if (c->ev_in) (void)hipEventDestroy(c->ev_in);
    if (c->ev_out) (void)hipEventDestroy(c->ev_out);
    if (c->side) (void)hipStreamDestroy(c->side);
    for (int s = 0; s < SL_NSLOTS; ++s) dev_free(c, c->slot_ptr[s]);
    if (c->pinned) (void)hipHostFree(c->pinned);
    for (hipEvent_t e : c->events) (void)hipEventDestroy(e);
    for (hipEvent_t e : c->prof_events) (void)hipEventDestroy(e);
    delete c;
    return ITE_OK;
}

const char* ite_last_error(const ite_ctx* c) { return c ? c->err.c_str() : "NULL context"; }

int ite_ctx_profile(ite_ctx* c, int enable) {
    if (!c) return ITE_EINVAL;
    return guarded(c, [&] {
        set_device(c);
        prof_collect(c);
        c->prof_on = enable != 0;
        if (c->prof_on)
            for (int k = 0; k < PK_COUNT; ++k) {
                c->prof_launches[k] = 0;
                c->prof_timed[k] = 0;
                c->prof_ms[k] = 0.0;
                c->prof_flops[k] = 0.0;
                c->prof_bytes[k] = 0.0;
            }
    });
}

int ite_ctx_profile_read(ite_ctx* c, long long* launches, double* ms, double* flops) {
    if (!c || !launches || !ms || !flops) return ITE_EINVAL;
    return guarded(c, [&] {
        set_device(c);
        prof_collect(c);
        *launches = c->prof_launches[PK_GEMM];
        *ms = c->prof_ms[PK_GEMM];
        *flops = c->prof_flops[PK_GEMM];
    });
}

int ite_ctx_profile_kernel(ite_ctx* c, int kind, long long* launches, long long* timed, double* ms_timed,
                           double* flops, double* bytes) {
    if (!c || !launches || !timed || !ms_timed || !flops || !bytes || kind < 0 || kind >= PK_COUNT)
        return ITE_EINVAL;
    return guarded(c, [&] {
        set_device(c);
        prof_collect(c);
        *launches = c->prof_launches[kind];
        *timed = c->prof_timed[kind];
        *ms_timed = c->prof_ms[kind];
        *flops = c->prof_flops[kind];
        *bytes = c->prof_bytes[kind];
    });
}

int ite_mpo_load(ite_ctx* c, int L, const int* d, const int* w, const double* const* W, ite_mpo** out) {
    if (!c || !out) return ITE_EINVAL;
    *out = nullptr;
    return guarded(c, [&] {
        set_device(c);
        *out = mpo_load(c, L, d, w, W);
    });
}

int ite_mpo_destroy(ite_mpo* m) {
    if (!m) return ITE_EINVAL;
    return guarded(m->ctx, [&] { mpo_destroy(m); });
}

int ite_mps_create(ite_ctx* c, int L, const int* d, const double* const* spinors, int chi_max, int pad_full,
                   ite_mps** out) {
    if (!c || !out) return ITE_EINVAL;
    *out = nullptr;
    return guarded(c, [&] {
        set_device(c);
        ITE_REQUIRE(spinors != nullptr, "mps_create: NULL spinors");
        ITE_REQUIRE(L >= 2 && d != nullptr, "mps_create: L must be >= 2");
        // normalised spinors
        std::vector<std::vector<double>> sp(L);
        for (int i = 0; i < L; ++i) {
            ITE_REQUIRE(d[i] >= 1 && d[i] <= 8, "mps_create: local dimension must be in 1..8");
            ITE_REQUIRE(spinors[i] != nullptr, "mps_create: NULL spinor");
            double nn = 0.0;
            for (int s = 0; s < d[i]; ++s) {
                ITE_REQUIRE(std::isfinite(spinors[i][s]), "mps_create: non-finite spinor entry");
                nn += spinors[i][s] * spinors[i][s];
            }
            ITE_REQUIRE(nn > 0.0, "mps_create: zero spinor");
            const double inv = 1.0 / std::sqrt(nn);
            sp[i].resize(d[i]);
            for (int s = 0; s < d[i]; ++s) sp[i][s] = spinors[i][s] * inv;
        }
        std::unique_ptr<ite_mps, void (*)(ite_mps*)> p(mps_new(c, L, d, chi_max), mps_destroy);
        if (pad_full) p->D = p->Dcap;
        for (int i = 0; i < L; ++i) {
            const int dl = p->D[i], dr = p->D[i + 1], di = d[i];
            const int cols = di * dr;
            // u = spinor (x) e_0 (index s * dr); rows of I - 2 v v^T / v.v with v = e_0 - u
            std::vector<double> u(cols, 0.0);
            for (int s = 0; s < di; ++s) u[(size_t)s * dr] = sp[i][s];
            std::vector<double> v(cols);
            for (int k = 0; k < cols; ++k) v[k] = (k == 0 ? 1.0 : 0.0) - u[k];
            double vv = 0.0;
            for (double x : v) vv += x * x;
            std::vector<double> A((size_t)dl * cols, 0.0);
            for (int r = 0; r < dl; ++r)
                for (int k = 0; k < cols; ++k) {
                    double val = (r == k) ? 1.0 : 0.0;
                    if (vv > 0.0) val -= 2.0 * v[r] * v[k] / vv;
                    A[(size_t)r * cols + k] = val;
                }
            h2d_wait(c, p->A[i], A.data(), A.size() * sizeof(double));
        }
        p->tau = 0.0;
        p->e_valid = false;
        *out = p.release();
    });
}

int ite_mps_load(ite_ctx* c, int L, const int* d, const int* chi, const double* const* A, int chi_max,
                 ite_mps** out) {
    if (!c || !out) return ITE_EINVAL;
    *out = nullptr;
    return guarded(c, [&] {
        set_device(c);
        ITE_REQUIRE(chi && A && d, "mps_load: NULL array");
        ITE_REQUIRE(L >= 2, "mps_load: L must be >= 2");
        ITE_REQUIRE(chi[0] == 1 && chi[L] == 1, "mps_load: boundary bond dimensions must be 1");
        std::unique_ptr<ite_mps, void (*)(ite_mps*)> p(mps_new(c, L, d, chi_max), mps_destroy);
        for (int i = 0; i <= L; ++i)
            ITE_REQUIRE(chi[i] >= 1 && chi[i] <= p->Dcap[i], "mps_load: bond dimension out of range");
        for (int i = 0; i < L; ++i) {
            ITE_REQUIRE(A[i] != nullptr, "mps_load: NULL tensor");
            const size_t n = (size_t)chi[i] * d[i] * chi[i + 1];
            for (size_t k = 0; k < n; ++k) ITE_REQUIRE(std::isfinite(A[i][k]), "mps_load: non-finite entry");
            h2d_wait(c, p->A[i], A[i], n * sizeof(double));
        }
        p->D.assign(chi, chi + L + 1);
        *out = p.release();
    });
}

int ite_mps_export(ite_mps* p, int* chi, double* const* A) {
    if (!p || !chi) return ITE_EINVAL;
    return guarded(p->ctx, [&] {
        set_device(p->ctx);
        for (int i = 0; i <= p->L; ++i) chi[i] = p->D[i];
        if (A) {
            sync(p->ctx);
            for (int i = 0; i < p->L; ++i) {
                ITE_REQUIRE(A[i] != nullptr, "mps_export: NULL buffer");
                d2h_wait(p->ctx, A[i], p->A[i], (size_t)p->D[i] * p->d[i] * p->D[i + 1] * sizeof(double));
            }
        }
    });
}

int ite_mps_destroy(ite_mps* p) {
    if (!p) return ITE_EINVAL;
    ite_ctx* c = p->ctx;
    return guarded(c, [&] {
        set_device(c);
        sync(c);
        mps_destroy(p);
    });
}

int ite_mps_get_tau(const ite_mps* p, double* tau) {
    if (!p || !tau) return ITE_EINVAL;
    *tau = p->tau;
    return ITE_OK;
}

int ite_mps_set_tau(ite_mps* p, double tau) {
    if (!p || !std::isfinite(tau) || tau < 0) return ITE_EINVAL;
    p->tau = tau;
    return ITE_OK;
}

int ite_imag_step(ite_mps* psi, const ite_mpo* H, double h, const ite_step_opts* o, ite_step_report* rep) {
    if (!psi || !H || !opts_ok(o)) return ITE_EINVAL;
    if (psi->ctx != H->ctx) return ITE_ESTATE;
    return guarded(psi->ctx, [&] {
        set_device(psi->ctx);
        imag_step(psi, H, h, *o, rep);
    });
}

int ite_gl_coefficients(int p, double* c, double* b, double* A, double* w, double* r_inf) {
    if (p < 1 || p > 7 || !c || !b || !A || !w || !r_inf) return ITE_EINVAL;
    try {
        const GlCoef g = gl_coefficients(p);
        std::copy(g.c.begin(), g.c.end(), c);
        std::copy(g.b.begin(), g.b.end(), b);
        std::copy(g.A.begin(), g.A.end(), A);
        std::copy(g.w.begin(), g.w.end(), w);
        *r_inf = g.r_inf;
    } catch (...) {
        return ITE_EINVAL;
    }
    return ITE_OK;
}

int ite_mpo_apply(const ite_mpo* O, ite_mps* psi, int chi_max, double cutoff, double tie_rel, ite_mps** out,
                  double* max_disc) {
    if (!O || !psi || !out) return ITE_EINVAL;
    *out = nullptr;
    if (psi->ctx != O->ctx) return ITE_ESTATE;
    return guarded(psi->ctx, [&] {
        set_device(psi->ctx);
        std::unique_ptr<ite_mps, void (*)(ite_mps*)> r(mps_new(psi->ctx, psi->L, psi->d.data(), psi->chi_max),
                                                      mps_destroy);
        const double disc = mpo_apply_dm(psi, O, chi_max, cutoff, tie_rel, r.get());
        if (max_disc) *max_disc = disc;
        *out = r.release();
    });
}

int ite_step_batch(ite_ctx* c, int n, ite_mps* const* psi, const ite_mpo* const* H, const double* h,
                   const ite_step_opts* const* opts, ite_step_report* reps, int* status) {
    if (!c || n < 1 || !psi || !H || !h || !opts) return ITE_EINVAL;
    int rc = guarded(c, [&] {
        set_device(c);
        for (int j = 0; j < n; ++j)
            if (!psi[j] || psi[j]->ctx != c) ITE_FAIL(psi[j] ? ITE_ESTATE : ITE_EINVAL, "step_batch: state not on ctx");
        step_batch(n, psi, H, h, opts, reps, status);
    });
    if (rc == ITE_OK && status)
        for (int j = 0; j < n; ++j)
            if (status[j] != ITE_OK) return status[j];
    return rc;
}

int ite_ctx_set_graphs(ite_ctx* c, int enable) {
    if (!c) return ITE_EINVAL;
    c->use_graphs = enable != 0;
    return ITE_OK;
}

int ite_ctx_batch_stats(ite_ctx* c, long long* solves, long long* captures, long long* replays) {
    if (!c) return ITE_EINVAL;
    if (solves) *solves = c->batch_solves;
    if (captures) *captures = c->graph_captures;
    if (replays) *replays = c->graph_replays;
    return ITE_OK;
}

int ite_dmrg_sweeps(ite_mps* psi, const ite_mpo* H, int nsweeps, int chi_max, double cutoff, double tie_rel,
                    int krylov_dim, int max_cycles, double tol, double* energy, double* max_res_rel,
                    double* max_disc, long long* matvecs) {
    if (!psi || !H) return ITE_EINVAL;
    if (psi->ctx != H->ctx) return ITE_ESTATE;
    if (nsweeps < 1 || max_cycles < 1 || krylov_dim < 1 || krylov_dim > 64 || chi_max < 1) return ITE_EINVAL;
    if (!(cutoff >= 0.0 && cutoff < 1.0) || !(tie_rel >= 0.0) || !(tol >= 0.0)) return ITE_EINVAL;
    return guarded(psi->ctx, [&] {
        set_device(psi->ctx);
        DmrgOpts o;
        o.nsweeps = nsweeps;
        o.chi_max = chi_max;
        o.cutoff = cutoff;
        o.tie_rel = tie_rel;
        o.krylov_dim = krylov_dim;
        o.max_cycles = max_cycles;
        o.tol = tol;
        DmrgReport r;
        dmrg_sweeps(psi, H, o, &r);
        if (energy) *energy = r.energy;
        if (max_res_rel) *max_res_rel = r.max_res_rel;
        if (max_disc) *max_disc = r.max_disc;
        if (matvecs) *matvecs = r.matvecs;
    });
}

int ite_mps_sample(ite_mps* psi, int nsamples, int L, const double* uniforms, int* configs) {
    if (!psi || !uniforms || !configs || nsamples < 1) return ITE_EINVAL;
    return guarded(psi->ctx, [&] {
        set_device(psi->ctx);
        ITE_REQUIRE(L == psi->L, "mps_sample: L differs from the state's length (buffers of nsamples * L entries)");
        mps_sample(psi, nsamples, uniforms, configs);
    });
}

int ite_mps_expect_site(ite_mps* psi, int site, const double* op, double* out) {
    if (!psi || !op || !out) return ITE_EINVAL;
    return guarded(psi->ctx, [&] {
        set_device(psi->ctx);
        *out = site_expect(psi, site, op);
    });
}

int ite_metts_chain(const ite_mpo* H, const int* start, int chi_max, double beta, double tau0, double ratio,
                    const ite_step_opts* opts, int site, const double* op, int nsamples, int L,
                    const double* uniforms, int* configs, double* energies, double* observables) {
    if (!H || !start || !opts || !op || !uniforms || !configs || !energies || !observables || nsamples < 1)
        return ITE_EINVAL;
    ite_ctx* c = H->ctx;
    int rc = guarded(c, [&] {
        ITE_REQUIRE(L == H->L, "metts_chain: L differs from the Hamiltonian's length");
        ITE_REQUIRE(std::isfinite(beta) && std::isfinite(tau0) && tau0 > 0.0 && 0.5 * beta > tau0,
                    "metts_chain: need 0 < tau0 < beta / 2");
        ITE_REQUIRE(site >= 0 && site < L, "metts_chain: site out of range");
        for (int i = 0; i < L; ++i)
            ITE_REQUIRE(start[i] >= 0 && start[i] < H->d[i], "metts_chain: start configuration out of range");
    });
    if (rc != ITE_OK) return rc;
    int n = 0;
    ite_loggrid(tau0, 0.5 * beta, ratio, nullptr, 0, &n);
    if (n < 2) {
        c->err = "metts_chain: bad grid (need ratio > 1)";
        return ITE_EINVAL;
    }
    std::vector<int> cfg(start, start + L);
    std::vector<ite_step_report> reps(n);
    std::vector<std::vector<double>> sp(L);
    std::vector<const double*> spp(L);
    for (int k = 0; k < nsamples; ++k) {
        for (int i = 0; i < L; ++i) {
            configs[(size_t)k * L + i] = cfg[i];
            sp[i].assign(H->d[i], 0.0);
            sp[i][cfg[i]] = 1.0;
            spp[i] = sp[i].data();
        }
        // |psi_k> ~ exp(-beta H / 2)|cfg> on the geometric grid tau0 -> beta / 2
        ite_mps* psi = nullptr;
        rc = ite_mps_create(c, L, H->d.data(), spp.data(), chi_max, 0, &psi);
        if (rc != ITE_OK) return rc;
        int steps = 0;
        rc = ite_evolve_loggrid(psi, H, tau0, 0.5 * beta, ratio, opts, reps.data(), n, &steps);
        if (rc == ITE_OK) {
            energies[k] = steps > 0 ? reps[steps - 1].energy : 0.0;
            rc = ite_mps_expect_site(psi, site, op, &observables[k]);
        }
        // collapse into the product basis: the next chain element
        if (rc == ITE_OK) rc = ite_mps_sample(psi, 1, L, uniforms + (size_t)k * L, cfg.data());
        ite_mps_destroy(psi);
        if (rc != ITE_OK) return rc;
    }
    return ITE_OK;
}

int ite_mps_sample_noalloc(ite_mps* psi, int nsamples, int L, const double* uniforms, int* configs) {
    if (!psi || !uniforms || !configs || nsamples < 1) return ITE_EINVAL;
    return guarded(psi->ctx, [&] {
        set_device(psi->ctx);
        ITE_REQUIRE(L == psi->L, "mps_sample_noalloc: L differs from the state's length");
        mps_sample_noalloc(psi, nsamples, uniforms, configs, noalloc_scratch(psi->ctx->device),
                           noalloc_scratch_doubles());
    });
}

int ite_loggrid(double tau0, double tau1, double ratio, double* out, int cap, int* n) {
    if (!n) return ITE_EINVAL;
    *n = 0;
    if (!(std::isfinite(tau0) && std::isfinite(tau1) && std::isfinite(ratio))) return ITE_EINVAL;
    if (!(tau0 > 0.0 && tau1 > tau0 && ratio > 1.0)) return ITE_EINVAL;
    int cnt = 2;
    double t = tau0;
    while (t < tau1) {
        t = std::min(t * ratio, tau1);
        ++cnt;
        if (cnt > 100000000) return ITE_EINVAL;
    }
    *n = cnt;
    if (!out || cap < cnt) return ITE_EINVAL;
    out[0] = 0.0;
    out[1] = tau0;
    t = tau0;
    for (int k = 2; k < cnt; ++k) {
        t = std::min(t * ratio, tau1);
        out[k] = t;
    }
    return ITE_OK;
}

int ite_panel_grid(double tau_max, int P, int n, double* out, int cap, int* npts) {
    if (!npts) return ITE_EINVAL;
    *npts = 0;
    if (!(std::isfinite(tau_max) && tau_max > 0.0) || P < 1 || n < 1 || P > 1000) return ITE_EINVAL;
    const int cnt = P * n + 1;
    *npts = cnt;
    if (!out || cap < cnt) return ITE_EINVAL;
    out[0] = 0.0;
    double a = 0.0;
    int k = 1;
    for (int j = 1; j <= P; ++j) {
        const double b = tau_max / std::ldexp(1.0, P - j);
        for (int i = 1; i <= n; ++i) out[k++] = a + (b - a) * i / n;
        a = b;
    }
    return ITE_OK;
}

static int evolve_points(ite_mps* psi, const ite_mpo* H, const double* taus, int n_taus, const ite_step_opts* o,
                         ite_step_report* per_step, int max_steps, int* n_steps) {
    if (n_steps) *n_steps = 0;
    int done = 0;
    int rc = guarded(psi->ctx, [&] {
        set_device(psi->ctx);
        for (int k = 1; k < n_taus; ++k)
            ITE_REQUIRE(std::isfinite(taus[k]) && taus[k] > taus[k - 1], "evolve: grid must increase");
        // first grid point after the current tau (with a relative slack for rounding)
        int k0 = 1;
        const double eps = 1e-12 * std::max(1.0, std::fabs(psi->tau));
        while (k0 < n_taus && taus[k0] <= psi->tau + eps) ++k0;
        for (int k = k0; k < n_taus; ++k) {
            const double tcur = k == k0 ? psi->tau : taus[k - 1];
            const double dtau = taus[k] - tcur;
            if (!(dtau > 0.0)) continue;
            const double h = o->scheme == ITE_SCHEME_TRAP ? 0.5 * dtau : dtau;
            ite_step_report rep{};
            imag_step(psi, H, h, *o, &rep);
            psi->tau = taus[k];   // exactly on the grid
            rep.tau = taus[k];
            if (per_step && done < max_steps) per_step[done] = rep;
            ++done;
            if (n_steps) *n_steps = done;
        }
    });
    if (n_steps) *n_steps = done;
    return rc;
}

int ite_evolve_loggrid(ite_mps* psi, const ite_mpo* H, double tau0, double tau1, double ratio,
                       const ite_step_opts* o, ite_step_report* per_step, int max_steps, int* n_steps) {
    if (!psi || !H || !o) return ITE_EINVAL;
    if (psi->ctx != H->ctx) return ITE_ESTATE;
    int n = 0;
    int rc = ite_loggrid(tau0, tau1, ratio, nullptr, 0, &n);
    if (n == 0) {
        psi->ctx->err = "evolve_loggrid: need 0 < tau0 < tau1 and ratio > 1";
        return rc;
    }
    std::vector<double> g(n);
    rc = ite_loggrid(tau0, tau1, ratio, g.data(), n, &n);
    if (rc != ITE_OK) return rc;
    return evolve_points(psi, H, g.data(), n, o, per_step, max_steps, n_steps);
}

int ite_evolve_grid(ite_mps* psi, const ite_mpo* H, const double* taus, int n_taus, const ite_step_opts* o,
                    ite_step_report* per_step, int max_steps, int* n_steps) {
    if (!psi || !H || !o || !taus || n_taus < 2) return ITE_EINVAL;
    if (psi->ctx != H->ctx) return ITE_ESTATE;
    return evolve_points(psi, H, taus, n_taus, o, per_step, max_steps, n_steps);
}

int ite_measure_energy(ite_mps* psi, const ite_mpo* H, double* E) {
    if (!psi || !H || !E) return ITE_EINVAL;
    if (psi->ctx != H->ctx) return ITE_ESTATE;
    return guarded(psi->ctx, [&] {
        set_device(psi->ctx);
        if (H->L != psi->L) ITE_FAIL(ITE_ESTATE, "measure_energy: MPS and MPO lengths differ");
        *E = measure_energy(psi, H);
        psi->energy = *E;
        psi->e_valid = true;
    });
}

int ite_mps_overlap(ite_mps* a, ite_mps* b, double* out) {
    if (!a || !b || !out) return ITE_EINVAL;
    if (a->ctx != b->ctx) return ITE_ESTATE;
    return guarded(a->ctx, [&] {
        set_device(a->ctx);
        if (a->L != b->L || a->d != b->d) ITE_FAIL(ITE_ESTATE, "overlap: different chains");
        *out = overlap(a, b);
    });
}

int ite_mps_norm(ite_mps* p, double* out) {
    if (!p || !out) return ITE_EINVAL;
    return guarded(p->ctx, [&] {
        set_device(p->ctx);
        const size_t n = (size_t)p->D[0] * p->d[0] * p->D[1];
        *out = std::sqrt(std::max(0.0, dot(p->ctx, p->A[0], p->A[0], n)));
    });
}

// ---- parity-test building blocks ------------------------------------------

int ite_debug_gemm(ite_ctx* c, int transA, int transB, int M, int N, int K, double alpha, const double* A, int lda,
                   const double* B, int ldb, double beta, const double* C, int ldc, double* D, int ldd, int prec) {
    if (!c) return ITE_EINVAL;
    return guarded(c, [&] {
        set_device(c);
        ITE_REQUIRE(M >= 0 && N >= 0 && K >= 0 && A && B && D, "debug_gemm: bad arguments");
        Gemm g;
        g.M = M; g.N = N; g.K = K; g.tA = transA != 0; g.tB = transB != 0;
        g.alpha = alpha; g.beta = beta; g.C = C; g.ldc = ldc; g.D = D; g.ldd = ldd;
        g.lda = lda; g.ldb = ldb;
        if (prec == ITE_PREC_FP64) {
            // the library's FP64 product dispatch (K parts for under-filled
            // outputs with a long K)
            gemm(c, g.tA, g.tB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, D, ldd);
        } else {
            const size_t na = (size_t)(transA ? K : M) * lda, nbb = (size_t)(transB ? N : K) * ldb;
            if (prec == ITE_PREC_FP32_IR) {
                float* a32 = slot_t<float>(c, SL_LO_L, na);
                float* b32 = slot_t<float>(c, SL_LO_R, nbb);
                convert_f32(A, a32, na, c->stream);
                convert_f32(B, b32, nbb, c->stream);
                g.A = a32; g.B = b32;
                gemm_f32(g, c->stream);
            } else if (prec == ITE_PREC_BF16_IR) {
                uint16_t* a16 = slot_t<uint16_t>(c, SL_LO_L, na);
                uint16_t* b16 = slot_t<uint16_t>(c, SL_LO_R, nbb);
                convert_bf16(A, a16, na, c->stream);
                convert_bf16(B, b16, nbb, c->stream);
                g.A = a16; g.B = b16;
                gemm_bf16(g, c->stream);
            } else {
                ITE_FAIL(ITE_EINVAL, "debug_gemm: unknown precision");
            }
        }
        sync(c);
    });
}

int ite_debug_heff_apply(ite_ctx* c, int Dxl, int Dyl, int Dxr, int Dyr, int d1, int d2, int w0, int w1, int w2,
                         const double* L, const double* W1h, const double* W2h, const double* R, const double* theta,
                         double alpha, double beta, double* y, int prec) {
    if (!c) return ITE_EINVAL;
    return guarded(c, [&] {
        set_device(c);
        ITE_REQUIRE(L && W1h && W2h && R && theta && y, "debug_heff_apply: NULL pointer");
        ITE_REQUIRE(Dxl > 0 && Dyl > 0 && Dxr > 0 && Dyr > 0 && d1 > 0 && d2 > 0 && w0 > 0 && w1 > 0 && w2 > 0,
                    "debug_heff_apply: bad shape");
        ITE_REQUIRE(alpha == 0.0 || (Dxl == Dyl && Dxr == Dyr), "debug_heff_apply: alpha needs square shapes");
        ITE_REQUIRE(prec >= 0 && prec <= 2, "debug_heff_apply: unknown precision");
        TmpCsr t(c, pair_matrix(W1h, W2h, w0, w1, w2, d1, d2), d1 * d2 * w2, w0 * d1 * d2);
        HeffShape s{Dxl, Dyl, Dxr, Dyr, d1, d2, w0, w2};
        heff_apply(c, s, L, t.cs, R, theta, beta, alpha, alpha != 0.0 ? theta : nullptr, y,
                   prec == 0 ? Prec::F64 : (prec == 1 ? Prec::F32 : Prec::BF16));
        sync(c);
    });
}

int ite_debug_heff_time(ite_ctx* c, int Dxl, int Dyl, int Dxr, int Dyr, int d1, int d2, int w0, int w1, int w2,
                        const double* L, const double* W1h, const double* W2h, const double* R, const double* theta,
                        double alpha, double beta, double* y, int prec, int reps, double* ms_per_product) {
    if (!c) return ITE_EINVAL;
    return guarded(c, [&] {
        set_device(c);
        ITE_REQUIRE(L && W1h && W2h && R && theta && y && ms_per_product, "debug_heff_time: NULL pointer");
        ITE_REQUIRE(Dxl > 0 && Dyl > 0 && Dxr > 0 && Dyr > 0 && d1 > 0 && d2 > 0 && w0 > 0 && w1 > 0 && w2 > 0,
                    "debug_heff_time: bad shape");
        ITE_REQUIRE(alpha == 0.0 || (Dxl == Dyl && Dxr == Dyr), "debug_heff_time: alpha needs square shapes");
        ITE_REQUIRE(prec >= 0 && prec <= 2, "debug_heff_time: unknown precision");
        ITE_REQUIRE(reps >= 1, "debug_heff_time: reps must be positive");
        TmpCsr t(c, pair_matrix(W1h, W2h, w0, w1, w2, d1, d2), d1 * d2 * w2, w0 * d1 * d2);
        HeffShape s{Dxl, Dyl, Dxr, Dyr, d1, d2, w0, w2};
        const Prec p = prec == 0 ? Prec::F64 : (prec == 1 ? Prec::F32 : Prec::BF16);
        const void* Llo = nullptr;
        const void* Rlo = nullptr;
        if (p != Prec::F64) lo_shadows(c, s, p, L, R, &Llo, &Rlo);
        auto once = [&] { heff_apply(c, s, L, t.cs, R, theta, beta, alpha, alpha != 0.0 ? theta : nullptr, y, p, Llo, Rlo); };
        once();
        hipEvent_t e0 = nullptr, e1 = nullptr;
        HIP_CHECK(hipEventCreate(&e0));
        HIP_CHECK(hipEventCreate(&e1));
        HIP_CHECK(hipEventRecord(e0, c->stream));
        for (int r = 0; r < reps; ++r) once();
        HIP_CHECK(hipEventRecord(e1, c->stream));
        HIP_CHECK(hipEventSynchronize(e1));
        float ms = 0.0f;
        HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        *ms_per_product = ms / reps;
    });
}

int ite_debug_env_update(ite_ctx* c, int dir, int Dxa, int Dya, int Dxb, int Dyb, int d, int wl, int wr,
                         const double* E, const double* X, const double* Wh, const double* Y, double* Eout) {
    if (!c) return ITE_EINVAL;
    return guarded(c, [&] {
        set_device(c);
        ITE_REQUIRE(E && X && Y && Eout, "debug_env_update: NULL pointer");
        ITE_REQUIRE(Dxa > 0 && Dya > 0 && Dxb > 0 && Dyb > 0 && d > 0 && wl > 0 && wr > 0,
                    "debug_env_update: bad shape");
        ITE_REQUIRE(dir == 0 || dir == 1, "debug_env_update: dir must be 0 or 1");
        if (!Wh) {
            if (dir == 0) {
                env_left(c, Dxa, Dya, Dxb, Dyb, d, 1, 1, E, X, nullptr, Y, Eout);
            } else {
                std::vector<double> Id((size_t)d * d, 0.0);
                for (int i = 0; i < d; ++i) Id[(size_t)i * d + i] = 1.0;
                TmpCsr t(c, Id, d, d);
                env_right_overlap_pub(c, t.cs, Dxa, Dya, Dxb, Dyb, d, E, X, Y, Eout);
            }
            sync(c);
            return;
        }
        std::vector<double> ML((size_t)d * wr * wl * d), MR((size_t)d * wl * wr * d);
        for (int a = 0; a < wl; ++a)
            for (int b = 0; b < wr; ++b)
                for (int p = 0; p < d; ++p)
                    for (int s = 0; s < d; ++s) {
                        const double v = Wh[(((size_t)a * wr + b) * d + p) * d + s];
                        ML[((size_t)p * wr + b) * (wl * d) + a * d + s] = v;
                        MR[((size_t)p * wl + a) * (wr * d) + b * d + s] = v;
                    }
        if (dir == 0) {
            TmpCsr t(c, ML, d * wr, wl * d);
            env_left(c, Dxa, Dya, Dxb, Dyb, d, wl, wr, E, X, &t.cs, Y, Eout);
            sync(c);
        } else {
            TmpCsr t(c, MR, d * wl, wr * d);
            env_right(c, Dxa, Dya, Dxb, Dyb, d, wl, wr, E, X, &t.cs, Y, Eout);
            sync(c);
        }
    });
}

int ite_debug_svd_split(ite_ctx* c, int dir, int Dl, int d1, int d2, int Dr, const double* theta, int chi_max,
                        double cutoff, double tie_rel, double* A1, double* A2, double* sigma_out, int* k_out,
                        double* disc_out) {
    if (!c) return ITE_EINVAL;
    return guarded(c, [&] {
        set_device(c);
        ITE_REQUIRE(theta && A1 && A2, "debug_svd_split: NULL pointer");
        ITE_REQUIRE(Dl > 0 && d1 > 0 && d2 > 0 && Dr > 0 && chi_max >= 1, "debug_svd_split: bad shape");
        ITE_REQUIRE(dir == 0 || dir == 1, "debug_svd_split: dir must be 0 or 1");
        std::vector<double> s;
        SplitResult r = split(c, dir, Dl, d1, d2, Dr, theta, chi_max, cutoff, tie_rel, A1, A2, &s);
        if (sigma_out) std::memcpy(sigma_out, s.data(), s.size() * sizeof(double));
        if (k_out) *k_out = r.k;
        if (disc_out) *disc_out = r.disc;
    });
}

int ite_debug_local_solve(ite_ctx* c, int Dl, int Dr, int d1, int d2, int w0, int w1, int w2, const double* L,
                          const double* W1h, const double* W2h, const double* R, double alpha, double beta,
                          const double* b, const double* x0, int krylov_dim, int max_cycles, double tol,
                          int precision, int max_refine, double tol_refine, double* x, int* matvecs,
                          double* res_rel) {
    if (!c) return ITE_EINVAL;
    return guarded(c, [&] {
        set_device(c);
        ITE_REQUIRE(L && W1h && W2h && R && b && x0 && x, "debug_local_solve: NULL pointer");
        ITE_REQUIRE(Dl > 0 && Dr > 0 && d1 > 0 && d2 > 0 && w0 > 0 && w1 > 0 && w2 > 0, "debug_local_solve: bad shape");
        ITE_REQUIRE(krylov_dim >= 1 && krylov_dim <= 64 && max_cycles >= 1, "debug_local_solve: bad budget");
        ITE_REQUIRE(precision >= 0 && precision <= 2 && max_refine >= 1, "debug_local_solve: bad precision options");
        TmpCsr t(c, pair_matrix(W1h, W2h, w0, w1, w2, d1, d2), d1 * d2 * w2, w0 * d1 * d2);
        LocalOp op;
        op.s = HeffShape{Dl, Dl, Dr, Dr, d1, d2, w0, w2};
        op.L = L;
        op.R = R;
        op.ww = &t.cs;
        op.alpha = alpha;
        op.beta = beta;
        const size_t n = op.n();
        HIP_CHECK(hipMemcpyAsync(x, x0, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        SolveStats st = local_solve(c, op, b, x, krylov_dim, max_cycles, tol, precision, max_refine, tol_refine);
        sync(c);
        if (matvecs) *matvecs = st.matvecs64 + st.matvecs_lo;
        if (res_rel) *res_rel = st.res_rel;
    });
}

int ite_debug_mfma_probe(ite_ctx* c, int kind, double* out) {
    if (!c || !out) return ITE_EINVAL;
    return guarded(c, [&] {
        set_device(c);
        ITE_REQUIRE(kind == 0, "debug_mfma_probe: unknown kind");
        double* d = slot_t<double>(c, SL_TMPA, 256);
        mfma_probe_f64(d, c->stream);
        HIP_CHECK(hipMemcpyAsync(out, d, 256 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        sync(c);
    });
}

}  // extern "C"
