// Steps built on the two-site sweep of one implicit step (imag_step_sweep):
//
//  * Gauss-Legendre collocation panels, the spectral variant of the Method
//    section: on a panel [a, a + dt] the solution is a polynomial of degree
//    p - 1 in tau whose values Y_i at the p Gauss-Legendre nodes satisfy the
//    integral form of the evolution equation (Eq. 2 from a):
//        (I + dt A (x) (H - s)) Y = 1 (x) psi(a),   A_ij = int_0^(c_i) l_j,
//    l_j the Lagrange polynomial of the nodes that is 1 at c_j.  The p node
//    values form one MPS on L + 1 sites whose first site indexes the node
//    (dimension p + 1, entry 0 holding psi(a)), so the system is one
//    backward-Euler-type solve (step dt, shift 0) with the augmented MPO
//    [[0, 0], [0, A]] (x) (H - s), the MPO of H - s being H's MPO in direct
//    sum with -s times the identity.  The end value follows from the stage
//    equations without another product: dt (H - s) Y = A^-1 (1 psi - Y), so
//    psi(a + dt) = psi - dt b^T (H - s) Y = r_inf psi + sum_j w_j Y_j with
//    w = A^-T b and r_inf = 1 - b^T A^-1 1 (the Pade approximant's value at
//    infinity); it is the node site contracted with (r_inf, w) into site 1.
//    The widened bonds near the left end are then cut back to the chain's
//    own by exact two-site splits (cutoff 0), left to right up to the last
//    bond above its capacity and back, so the panel leaves a right-
//    orthonormal state with the centre on site 1, as every step does.
//
//  * The trapezoid step with its right-hand side b = (I - h (H - s)) psi
//    formed as an MPS by the "density matrix" MPO-MPS product (Appendix B),
//    then (I + h (H - s)) x = b solved by the sweep in its backward-Euler
//    form with b in place of psi, x starting as b.
//
// The density-matrix product phi = O psi, with F_j the left environments of
// <phi|phi> (no truncation) and C_(j+1) what is already kept right of site j:
//    F_(j+1)[a', w', w, a] = sum F_j[c', v', v, c] psi_j[c', t', a']
//                            O_j[v', w', s, t'] O_j[v, w, s, t] psi_j[c, t, a]
//    T_j[a, w, s, k]       = sum psi_j[a, t, a2] O_j[w, w2, s, t] C_(j+1)[a2, w2, k]
//    rho_j[(s' k'), (s k)] = sum T_j[a', w', s', k'] F_j[a', w', w, a] T_j[a, w, s, k]
// The eigenvectors of rho_j's largest eigenvalues (their square roots are
// phi's singular values at bond j) are the rows of the new site tensor and
// C_j = T_j V; site 1 keeps T_1 whole.  Every contraction is an FP64 GEMM or
// a sparse MPO stage; the eigenvectors come from the one-sided Jacobi split
// of rho_j (for a symmetric positive semi-definite matrix the right singular
// vectors are eigenvectors and the singular values the eigenvalues).
#include "engine.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <memory>

namespace ite {

namespace {

struct MpoDel {
    void operator()(ite_mpo* m) const { mpo_destroy(m); }
};
using MpoPtr = std::unique_ptr<ite_mpo, MpoDel>;

// Gauss-Legendre nodes c (ascending) and weights b on [0, 1]: the roots of
// the Legendre polynomial P_p by Newton's method, P_p and P_(p-1) from the
// three-term recurrence (n + 1) P_(n+1) = (2n + 1) x P_n - n P_(n-1), the
// weights 2 / ((1 - x^2) P_p'(x)^2) on [-1, 1], mapped to [0, 1].
void gauss_legendre(int p, std::vector<double>& c, std::vector<double>& b) {
    c.assign(p, 0.0);
    b.assign(p, 0.0);
    auto legendre = [p](double x, double* P, double* dP) {
        double p0 = 1.0, p1 = x;
        for (int n = 1; n < p; ++n) {
            const double p2 = ((2.0 * n + 1.0) * x * p1 - n * p0) / (n + 1.0);
            p0 = p1;
            p1 = p2;
        }
        *P = p1;
        *dP = p * (x * p1 - p0) / (x * x - 1.0);
    };
    for (int k = 0; k < p; ++k) {
        double x = std::cos(M_PI * (k + 0.75) / (p + 0.5));
        double P = 0.0, dP = 1.0;
        for (int it = 0; it < 100; ++it) {
            legendre(x, &P, &dP);
            const double dx = P / dP;
            x -= dx;
            if (std::fabs(dx) <= 1e-16) break;
        }
        legendre(x, &P, &dP);
        // roots come out descending in x; store ascending in c
        c[p - 1 - k] = 0.5 * (1.0 + x);
        b[p - 1 - k] = 1.0 / ((1.0 - x * x) * dP * dP);
    }
}

// Solve M z = r for a small dense p x p matrix (row-major) by Gaussian
// elimination with partial pivoting.
std::vector<double> small_solve(std::vector<double> M, std::vector<double> r, int p) {
    for (int k = 0; k < p; ++k) {
        int piv = k;
        for (int i = k + 1; i < p; ++i)
            if (std::fabs(M[(size_t)i * p + k]) > std::fabs(M[(size_t)piv * p + k])) piv = i;
        if (piv != k) {
            for (int j = 0; j < p; ++j) std::swap(M[(size_t)k * p + j], M[(size_t)piv * p + j]);
            std::swap(r[k], r[piv]);
        }
        const double dkk = M[(size_t)k * p + k];
        if (!(std::fabs(dkk) > 0.0)) ITE_FAIL(ITE_EINVAL, "collocation matrix is singular");
        for (int i = k + 1; i < p; ++i) {
            const double f = M[(size_t)i * p + k] / dkk;
            for (int j = k; j < p; ++j) M[(size_t)i * p + j] -= f * M[(size_t)k * p + j];
            r[i] -= f * r[k];
        }
    }
    for (int k = p - 1; k >= 0; --k) {
        double acc = r[k];
        for (int j = k + 1; j < p; ++j) acc -= M[(size_t)k * p + j] * r[j];
        r[k] = acc / M[(size_t)k * p + k];
    }
    return r;
}

}  // namespace

GlCoef gl_coefficients(int p) {
    GlCoef g;
    g.p = p;
    gauss_legendre(p, g.c, g.b);
    auto lag = [&](int j, double x) {
        double v = 1.0;
        for (int m = 0; m < p; ++m)
            if (m != j) v *= (x - g.c[m]) / (g.c[j] - g.c[m]);
        return v;
    };
    // int_0^(c_i) l_j = c_i sum_k b_k l_j(c_i c_k): the p-point rule is exact
    // for the degree p - 1 polynomial l_j
    g.A.assign((size_t)p * p, 0.0);
    for (int i = 0; i < p; ++i)
        for (int j = 0; j < p; ++j) {
            double acc = 0.0;
            for (int k = 0; k < p; ++k) acc += g.b[k] * lag(j, g.c[i] * g.c[k]);
            g.A[(size_t)i * p + j] = g.c[i] * acc;
        }
    std::vector<double> At((size_t)p * p);
    for (int i = 0; i < p; ++i)
        for (int j = 0; j < p; ++j) At[(size_t)j * p + i] = g.A[(size_t)i * p + j];
    g.w = small_solve(At, g.b, p);
    const std::vector<double> z = small_solve(g.A, std::vector<double>(p, 1.0), p);
    double bz = 0.0;
    for (int i = 0; i < p; ++i) bz += g.b[i] * z[i];
    g.r_inf = 1.0 - bz;
    return g;
}

namespace {

// Host tensors of the direct sum of H's MPO (first site scaled by `ah`) with
// the identity MPO scaled by `ai` on the first site: the MPO of ah H + ai I,
// bond dimensions w + 1 inside the chain.
void direct_sum_identity(const ite_mpo* H, double ah, double ai, std::vector<std::vector<double>>& T,
                         std::vector<int>& wo) {
    const int L = H->L;
    T.assign(L, {});
    wo.assign(L + 1, 1);
    for (int i = 1; i < L; ++i) wo[i] = H->w[i] + 1;
    for (int i = 0; i < L; ++i) {
        const int wl = H->w[i], wr = H->w[i + 1], d = H->d[i];
        const int nl = wo[i], nr = wo[i + 1];
        std::vector<double>& t = T[i];
        t.assign((size_t)nl * nr * d * d, 0.0);
        auto at = [&](int a, int b2, int p, int s) -> double& { return t[(((size_t)a * nr + b2) * d + p) * d + s]; };
        auto W = [&](int a, int b2, int p, int s) { return H->Wh[i][(((size_t)a * wr + b2) * d + p) * d + s]; };
        const double sc = i == 0 ? ah : 1.0;
        for (int a = 0; a < wl; ++a)
            for (int b2 = 0; b2 < wr; ++b2)
                for (int p = 0; p < d; ++p)
                    for (int s = 0; s < d; ++s) at(a, b2, p, s) = sc * W(a, b2, p, s);
        // the identity channel: enters at the first site, closes at the last
        const int ia = i == 0 ? 0 : wl, ib = i == L - 1 ? 0 : wr;
        const double v = i == 0 ? ai : 1.0;
        for (int p = 0; p < d; ++p) at(ia, ib, p, p) += v;
    }
}

MpoPtr load_host_mpo(ite_ctx* c, const std::vector<int>& d, const std::vector<int>& w,
                     const std::vector<std::vector<double>>& T) {
    std::vector<const double*> ptrs(T.size());
    for (size_t i = 0; i < T.size(); ++i) ptrs[i] = T[i].data();
    return MpoPtr(mpo_load(c, (int)T.size(), d.data(), w.data(), ptrs.data()));
}

// The auxiliary state of psi with L sites of dimensions d (reallocated when
// the shape changes).
ite_mps* ensure_aux(ite_mps* psi, int L, const std::vector<int>& d) {
    ite_mps* a = psi->aux;
    if (a && a->L == L && a->d == d && a->chi_max == psi->chi_max) return a;
    mps_destroy(a);
    psi->aux = nullptr;
    psi->aux = mps_new(psi->ctx, L, d.data(), psi->chi_max);
    return psi->aux;
}

// Widen the bonds of the augmented state that are complete within chi and
// above the chain's own complete bond to complete, the others to at least
// what the node rank needs to pass (the
// node site first, of dimension p + 1; every other site right-orthonormal;
// a bond at most d_i times the widened bond right of site i): right to left, a
// widened right bond gets zero columns and a widened left bond the trailing
// rows of Q^T for the Householder QR of the site's rows transposed (an
// orthonormal completion of its rows).  The added basis states carry no
// weight: the same state, still right-orthonormal.
void widen_augmented(ite_ctx* c, ite_mps* a, int chi) {
    const int n = a->L;
    // what the node rank needs at each bond to pass: p + 1 over the
    // dimensions between
    std::vector<int> need(n + 1, 1);
    need[1] = a->d[0];
    for (int k = 2; k < n; ++k) need[k] = (need[k - 1] + a->d[k - 1] - 1) / a->d[k - 1];
    std::vector<int> tgt(n + 1);
    for (int k = 0; k <= n; ++k) {
        double left = 1.0, right = 1.0;
        for (int i = 0; i < k; ++i) left *= a->d[i];
        for (int i = k; i < n; ++i) right *= a->d[i];
        const double complete = std::min(left, right);
        // the chain's own complete bond (the node's dimension left out of
        // the left product): towards the right end the two are the same
        const double own = k == 0 ? 1.0 : std::min(left / a->d[0], right);
        tgt[k] = complete <= (double)chi && complete > own ? (int)complete
                                                           : std::max(a->D[k], std::min(need[k], chi));
        tgt[k] = std::min(std::max(tgt[k], a->D[k]), a->Dcap[k]);
    }
    // a site's rows can be completed only within d_i times its right bond
    for (int k = n - 1; k >= 1; --k) tgt[k] = std::max(a->D[k], std::min(tgt[k], a->d[k] * tgt[k + 1]));
    const std::vector<int> D0 = a->D;   // the tensors' shapes before widening
    for (int i = n - 1; i >= 0; --i) {
        const int Dl = D0[i], di = a->d[i], Dr = D0[i + 1];
        const int Tl = i == 0 ? Dl : tgt[i], Tr = tgt[i + 1];
        if (Tl == Dl && Tr == Dr) continue;
        const size_t ncol = (size_t)di * Tr;
        double* w = slot_t<double>(c, SL_TPSI, (size_t)Tl * ncol);
        // the site's rows with zero columns for the widened right bond
        fill(w, 0.0, (size_t)Tl * ncol, c->stream);
        HIP_CHECK(hipMemcpy2DAsync(w, sizeof(double) * Tr, a->A[i], sizeof(double) * Dr, sizeof(double) * Dr,
                                   (size_t)Dl * di, hipMemcpyDeviceToDevice, c->stream));
        if (Tl > Dl) {
            // Z = [R^T | I] -> Q^T Z; rows Dl.. of Q^T complete R's rows
            const int pz = (int)ncol, qz = Dl, ldz = pz + qz;
            ITE_REQUIRE(pz <= 2048, "gl panel: bond widening beyond 2048 rows");
            double* Z = slot_t<double>(c, SL_Z, (size_t)pz * ldz);
            double* ws = slot_t<double>(c, SL_QR, householder_workspace(pz, qz, ldz));
            jacobi_input(w, Dl, pz, 1, Z, c->stream);
            householder_rows(Z, pz, qz, ldz, ws, c->stream);
            HIP_CHECK(hipMemcpy2DAsync(w + (size_t)Dl * ncol, sizeof(double) * ncol, Z + (size_t)Dl * ldz + qz,
                                       sizeof(double) * ldz, sizeof(double) * ncol, (size_t)(Tl - Dl),
                                       hipMemcpyDeviceToDevice, c->stream));
        }
        d2d(c, a->A[i], w, (size_t)Tl * ncol);
    }
    tgt[0] = D0[0];
    a->D = tgt;
}

// Milliseconds since t0 after the context's stream has drained.
double ms_since(ite_ctx* c, std::chrono::steady_clock::time_point t0) {
    sync(c);
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

double step_shift(ite_mps* psi, const ite_mpo* H, const ite_step_opts& o) {
    if (o.shift_mode != ITE_SHIFT_TRACK) return o.shift;
    if (!psi->e_valid) {
        psi->energy = measure_energy(psi, H);
        psi->e_valid = true;
    }
    return psi->energy;
}

// ---------------------------------------------------------------------------
// Gauss-Legendre panel
// ---------------------------------------------------------------------------

void gl_panel(ite_mps* psi, const ite_mpo* H, double dt, const ite_step_opts& o, ite_step_report* rep) {
    ite_ctx* c = psi->ctx;
    const int L = psi->L, p = o.gl_nodes;
    const std::vector<int>& d = psi->d;
    const double s = step_shift(psi, H, o);
    const GlCoef g = gl_coefficients(p);
    // augmented MPO: node site [[0, 0], [0, A]], then the MPO of H - s
    std::vector<std::vector<double>> Ts;
    std::vector<int> ws;
    direct_sum_identity(H, 1.0, -s, Ts, ws);
    std::vector<std::vector<double>> Ta(L + 1);
    std::vector<int> da(L + 1), wa(L + 2);
    da[0] = p + 1;
    Ta[0].assign((size_t)(p + 1) * (p + 1), 0.0);
    for (int i = 0; i < p; ++i)
        for (int j = 0; j < p; ++j) Ta[0][(size_t)(i + 1) * (p + 1) + (j + 1)] = g.A[(size_t)i * p + j];
    wa[0] = 1;
    for (int i = 0; i < L; ++i) {
        da[i + 1] = d[i];
        Ta[i + 1] = std::move(Ts[i]);
        wa[i + 1] = ws[i];
    }
    wa[L + 1] = 1;
    MpoPtr Ha = load_host_mpo(c, da, wa, Ta);
    // augmented state: (1, .., 1) / sqrt(p + 1) on the node site, then psi
    ite_mps* aug = ensure_aux(psi, L + 1, da);
    aug->D.assign(L + 2, 1);
    fill(aug->A[0], 1.0 / std::sqrt((double)(p + 1)), (size_t)(p + 1), c->stream);
    for (int i = 0; i < L; ++i) {
        aug->D[i + 2] = psi->D[i + 1];
        d2d(c, aug->A[i + 1], psi->A[i], (size_t)psi->D[i] * d[i] * psi->D[i + 1]);
    }
    aug->tau = 0.0;
    aug->e_valid = false;
    // the node bond needs rank p + 1, and the sweep's first block can give
    // it at most d_1 D_2 with psi's bonds: then the bonds complete within
    // chi_max are widened first (the same state)
    const int chi_w = std::min(o.chi_max, psi->chi_max);
    if (p + 1 > d[0] * psi->D[1]) widen_augmented(c, aug, chi_w);
    ite_step_opts oa = o;
    oa.scheme = ITE_SCHEME_BE;
    oa.shift_mode = ITE_SHIFT_FIXED;
    oa.shift = 0.0;
    oa.rhs_mode = ITE_RHS_PROJECT;
    ite_step_report r{};
    imag_step_sweep(aug, Ha.get(), dt, oa, &r);
    const int aux_max = *std::max_element(aug->D.begin(), aug->D.end());
    const auto t_end = std::chrono::steady_clock::now();
    // end value: the node site contracted with (r_inf, w) into site 1
    const int D1 = aug->D[1], D2 = aug->D[2];
    double* sm = slot_t<double>(c, SL_DMC, (size_t)64 + D1 + (size_t)d[0] * D2);
    double* vdev = sm;
    double* rvec = sm + 32;
    double* a1 = sm + 32 + ((D1 + 31) & ~31);
    double* hv = pinned(c, 64);
    hv[0] = g.r_inf;
    for (int j = 0; j < p; ++j) hv[1 + j] = g.w[j];
    h2d(c, vdev, hv, sizeof(double) * (p + 1));
    gemm(c, false, false, 1, D1, p + 1, 1.0, vdev, p + 1, aug->A[0], D1, 0.0, nullptr, 0, rvec, D1);
    gemm(c, false, false, 1, d[0] * D2, D1, 1.0, rvec, D1, aug->A[1], (long)d[0] * D2, 0.0, nullptr, 0, a1,
         (long)d[0] * D2);
    d2d(c, aug->A[1], a1, (size_t)d[0] * D2);
    sync(c);   // the pinned staging buffer is reused by the next call
    // the chain: sites aug->A[1..L], bonds 1, aug->D[2..L+1]
    std::vector<double*> ch(aug->A.begin() + 1, aug->A.end());
    std::vector<int> cd(L + 1);
    cd[0] = 1;
    for (int b2 = 1; b2 <= L; ++b2) cd[b2] = aug->D[b2 + 1];
    const int chi = std::min(o.chi_max, psi->chi_max);
    const std::vector<int> caps = bond_caps(L, d, chi);
    int last = 0;
    for (int b2 = 1; b2 < L; ++b2)
        if (cd[b2] > caps[b2]) last = b2;
    auto cut = [&](int i, int dir) {
        const size_t n = (size_t)cd[i] * d[i] * d[i + 1] * cd[i + 2];
        double* th = slot_t<double>(c, SL_TPSI, n);
        two_site(c, cd[i], d[i], cd[i + 1], d[i + 1], cd[i + 2], ch[i], ch[i + 1], th);
        SplitResult sp = split(c, dir, cd[i], d[i], d[i + 1], cd[i + 2], th, std::min(chi, caps[i + 1]), 0.0,
                               o.tie_rel, ch[i], ch[i + 1], nullptr);
        cd[i + 1] = sp.k;
    };
    for (int i = 0; i < last; ++i) cut(i, 0);
    for (int i = last - 1; i >= 0; --i) cut(i, 1);
    const size_t n0 = (size_t)cd[0] * d[0] * cd[1];
    const double nrm = std::sqrt(std::max(0.0, dot(c, ch[0], ch[0], n0)));
    if (!(std::isfinite(nrm) && nrm > 0.0)) ITE_FAIL(ITE_ENONFINITE, "gl panel: non-finite state; psi left unchanged");
    scale(ch[0], 1.0 / nrm, n0, c->stream);
    for (int i = 0; i < L; ++i) d2d(c, psi->A[i], ch[i], (size_t)cd[i] * d[i] * cd[i + 1]);
    psi->D = cd;
    const double E = measure_energy(psi, H);
    if (!std::isfinite(E)) ITE_FAIL(ITE_ENONFINITE, "gl panel: non-finite energy");
    psi->tau += dt;
    psi->energy = E;
    psi->e_valid = true;
    r.tau = psi->tau;
    r.dtau = dt;
    r.h = dt;
    r.shift = s;
    r.energy = E;
    r.norm_before = nrm;
    r.max_chi = *std::max_element(cd.begin(), cd.end());
    r.aux_max_chi = aux_max;
    r.rhs_disc = 0.0;
    // the read-off and the cut back to the chain's bonds count as split time
    const double ms_end = ms_since(c, t_end);
    r.ms_split += ms_end;
    r.ms_total += ms_end;
    if (rep) *rep = r;
}

// ---------------------------------------------------------------------------
// Density-matrix MPO-MPS product
// ---------------------------------------------------------------------------

// CSR matrices of the product's MPO stages, per site j (w = O's bonds):
//   tmap: (t, w_(j+1)) -> (w_j, s)       T_j from psi_j C_(j+1)
//   kmap: (v, t) -> (s, w)               ket side of F_(j+1)
//   bmap: (v', s) -> (t', w')            bra side of F_(j+1)
//   ident: identity of size w_j          the (a, w) -> (w, a) transpose of T_j
struct DmMaps {
    ite_ctx* c = nullptr;
    std::vector<CsrDev> tmap, kmap, bmap, ident;
    void* block = nullptr;
    ~DmMaps() { dev_free(c, block); }
};

void build_dm_maps(ite_ctx* c, const ite_mpo* O, DmMaps& m) {
    const int L = O->L;
    std::vector<CsrHost> hs;
    for (int j = 0; j < L; ++j) {
        const int wl = O->w[j], wr = O->w[j + 1], d = O->d[j];
        auto W = [&](int a, int b2, int p, int s) { return O->Wh[j][(((size_t)a * wr + b2) * d + p) * d + s]; };
        std::vector<double> Mt((size_t)wl * d * d * wr, 0.0), Mk((size_t)d * wr * wl * d, 0.0),
            Mb((size_t)d * wr * wl * d, 0.0), Id((size_t)wl * wl, 0.0);
        for (int a = 0; a < wl; ++a)
            for (int b2 = 0; b2 < wr; ++b2)
                for (int s = 0; s < d; ++s)
                    for (int t = 0; t < d; ++t) {
                        const double v = W(a, b2, s, t);
                        Mt[((size_t)a * d + s) * (d * wr) + t * wr + b2] = v;      // (w s) <- (t w2)
                        Mk[((size_t)s * wr + b2) * (wl * d) + a * d + t] = v;      // (s w) <- (v t)
                        Mb[((size_t)t * wr + b2) * (wl * d) + a * d + s] = v;      // (t' w') <- (v' s)
                    }
        for (int a = 0; a < wl; ++a) Id[(size_t)a * wl + a] = 1.0;
        hs.push_back(dense_to_csr(Mt, wl * d, d * wr));
        hs.push_back(dense_to_csr(Mk, d * wr, wl * d));
        hs.push_back(dense_to_csr(Mb, d * wr, wl * d));
        hs.push_back(dense_to_csr(Id, wl, wl));
    }
    m.c = c;
    std::vector<CsrDev> dv = upload_csr(c, hs, &m.block);
    for (int j = 0; j < L; ++j) {
        m.tmap.push_back(dv[4 * j]);
        m.kmap.push_back(dv[4 * j + 1]);
        m.bmap.push_back(dv[4 * j + 2]);
        m.ident.push_back(dv[4 * j + 3]);
    }
}

}  // namespace

double mpo_apply_dm(ite_mps* psi, const ite_mpo* O, int chi_max, double cutoff, double tie_rel, ite_mps* out) {
    ite_ctx* c = psi->ctx;
    const int L = psi->L;
    if (O->L != L || O->d != psi->d) ITE_FAIL(ITE_ESTATE, "mpo_apply: MPO and MPS shapes differ");
    if (out->L != L || out->d != psi->d) ITE_FAIL(ITE_ESTATE, "mpo_apply: output has another shape");
    ITE_REQUIRE(chi_max >= 1, "mpo_apply: chi_max must be >= 1");
    ITE_REQUIRE(cutoff >= 0.0 && cutoff < 1.0, "mpo_apply: cutoff must be in [0, 1)");
    ITE_REQUIRE(tie_rel >= 0.0, "mpo_apply: tie_rel must be >= 0");
    const std::vector<int>& d = psi->d;
    const std::vector<int>& D = psi->D;
    const std::vector<int>& w = O->w;
    for (int j = 0; j < L; ++j)
        if (w[j] * d[j] > 128 || w[j + 1] * d[j] > 128)
            ITE_FAIL(ITE_EINVAL, "mpo_apply: more than 128 MPO-index x local-dimension inputs at a site");
    const int chi = std::min(chi_max, out->chi_max);
    const std::vector<int> caps = bond_caps(L, d, chi);
    DmMaps maps;
    build_dm_maps(c, O, maps);
    // left environments of <phi|phi>: F_j [D_j][w_j][w_j][D_j]
    std::vector<size_t> foff(L + 1, 0);
    for (int j = 0; j < L; ++j) foff[j + 1] = foff[j] + (size_t)D[j] * w[j] * w[j] * D[j];
    double* F = slot_t<double>(c, SL_DMF, foff[L]);
    fill(F, 1.0, 1, c->stream);
    for (int j = 0; j + 1 < L; ++j) {
        const int Dc = D[j], Da = D[j + 1], wv = w[j], ww = w[j + 1], dd = d[j];
        const size_t n1 = (size_t)Dc * wv * wv * dd * Da, n2 = (size_t)Dc * wv * dd * ww * Da,
                     n3 = (size_t)Dc * dd * ww * ww * Da;
        double* X1 = slot_t<double>(c, SL_DM1, n1);
        double* X2 = slot_t<double>(c, SL_DM2, n2);
        double* X3 = slot_t<double>(c, SL_DM3, n3);
        // X1[(c' v' v), (t a)] = F_j[(c' v' v), c] psi_j[c, (t a)]
        gemm(c, false, false, Dc * wv * wv, dd * Da, Dc, 1.0, F + foff[j], Dc, psi->A[j], (long)dd * Da, 0.0,
             nullptr, 0, X1, (long)dd * Da);
        // X2[(c' v')][(s w)][a] = sum_(v t) O[v, w, s, t] X1[(c' v')][(v t)][a]
        Stage st;
        st.G = Dc * wv; st.C = Da;
        st.in = X1; st.in_gs = (long)wv * dd * Da; st.in_s1 = Da;
        st.out = X2; st.out_gs = (long)dd * ww * Da; st.out_s1 = Da;
        stage(c, maps.kmap[j], st);
        // X3[c'][(t' w')][(w a)] = sum_(v' s) O[v', w', s, t'] X2[c'][(v' s)][(w a)]
        Stage sb;
        sb.G = Dc; sb.C = ww * Da;
        sb.in = X2; sb.in_gs = (long)wv * dd * ww * Da; sb.in_s1 = (long)ww * Da;
        sb.out = X3; sb.out_gs = (long)dd * ww * ww * Da; sb.out_s1 = (long)ww * Da;
        stage(c, maps.bmap[j], sb);
        // F_(j+1)[a', (w' w a)] = psi_j[(c' t'), a']^T X3[(c' t'), (w' w a)]
        gemm(c, true, false, Da, ww * ww * Da, Dc * dd, 1.0, psi->A[j], Da, X3, (long)ww * ww * Da, 0.0, nullptr, 0,
             F + foff[j + 1], (long)ww * ww * Da);
    }
    // from the right: T_j, rho_j, the kept eigenvectors
    std::vector<int> K(L + 1, 1);
    size_t cmax = 1;
    for (int j = 0; j <= L; ++j) cmax = std::max(cmax, (size_t)D[j] * w[j] * caps[j]);
    double* Cb = slot_t<double>(c, SL_DMC, 2 * cmax + 64);
    double* Ccur = Cb;
    double* Cnew = Cb + cmax + 32;
    fill(Ccur, 1.0, 1, c->stream);
    double disc = 0.0;
    std::vector<double> lam;
    for (int j = L - 1; j >= 0; --j) {
        const int Dj = D[j], Dn = D[j + 1], wj = w[j], wn = w[j + 1], dd = d[j], Kn = K[j + 1];
        const int nk = dd * Kn;
        double* P = slot_t<double>(c, SL_DM1, (size_t)Dj * dd * wn * Kn);
        double* T = slot_t<double>(c, SL_DM2, (size_t)Dj * wj * nk);
        // P[(a t), (w2 k)] = psi_j[(a t), a2] C[a2, (w2 k)]
        gemm(c, false, false, Dj * dd, wn * Kn, Dn, 1.0, psi->A[j], Dn, Ccur, (long)wn * Kn, 0.0, nullptr, 0, P,
             (long)wn * Kn);
        // T[a][(w s)][k] = sum_(t w2) O[w, w2, s, t] P[a][(t w2)][k]
        Stage st;
        st.G = Dj; st.C = Kn;
        st.in = P; st.in_gs = (long)dd * wn * Kn; st.in_s1 = Kn;
        st.out = T; st.out_gs = (long)wj * dd * Kn; st.out_s1 = Kn;
        stage(c, maps.tmap[j], st);
        if (j == 0) {
            d2d(c, out->A[0], T, (size_t)nk);
            K[0] = 1;
            break;
        }
        // T transposed to [w][a][(s k)]
        double* Twa = slot_t<double>(c, SL_DM3, (size_t)Dj * wj * nk);
        Stage sp;
        sp.G = Dj; sp.C = nk;
        sp.in = T; sp.in_gs = (long)wj * nk; sp.in_s1 = nk;
        sp.out = Twa; sp.out_gs = nk; sp.out_s1 = (long)Dj * nk;
        stage(c, maps.ident[j], sp);
        // G1[(a' w'), (s k)] = F_j[(a' w'), (w a)] Twa[(w a), (s k)]
        double* G1 = slot_t<double>(c, SL_DM1, (size_t)Dj * wj * nk);
        gemm(c, false, false, Dj * wj, nk, wj * Dj, 1.0, F + foff[j], (long)wj * Dj, Twa, nk, 0.0, nullptr, 0, G1,
             nk);
        // rho[(s' k'), (s k)] = T[(a' w'), (s' k')]^T G1[(a' w'), (s k)]
        double* rho = slot_t<double>(c, SL_DMR, (size_t)nk * nk);
        gemm(c, true, false, nk, nk, Dj * wj, 1.0, T, nk, G1, nk, 0.0, nullptr, 0, rho, nk);
        // eigenvectors: rows of V^T from the split of rho (no truncation there)
        const int kcap = std::min(chi, caps[j]);
        const int kall = std::min(nk, kcap);
        double* Vt = slot_t<double>(c, SL_DMV, (size_t)kall * nk);
        double* US = slot_t<double>(c, SL_DMU, (size_t)kall * nk);
        split(c, 1, nk, 1, 1, nk, rho, kall, 0.0, 0.0, US, Vt, &lam);
        std::vector<double> sq(lam.size());
        double total = 0.0;
        for (size_t i = 0; i < lam.size(); ++i) {
            sq[i] = std::sqrt(std::max(lam[i], 0.0));
            total += std::max(lam[i], 0.0);
        }
        const int kk = std::min(kall, truncation_rank(sq, cutoff, kcap, tie_rel));
        double dropped = 0.0;
        for (size_t i = kk; i < lam.size(); ++i) dropped += std::max(lam[i], 0.0);
        if (total > 0.0) disc = std::max(disc, dropped / total);
        // site j of phi: the kept rows [kk][s][k]; C_j[(a w), kk] = T V
        d2d(c, out->A[j], Vt, (size_t)kk * nk);
        gemm(c, false, true, Dj * wj, kk, nk, 1.0, T, nk, Vt, nk, 0.0, nullptr, 0, Cnew, kk);
        std::swap(Ccur, Cnew);
        K[j] = kk;
    }
    const size_t n0 = (size_t)d[0] * K[1];
    const double nrm2 = dot(c, out->A[0], out->A[0], n0);
    if (!(std::isfinite(nrm2) && nrm2 > 0.0)) ITE_FAIL(ITE_ENONFINITE, "mpo_apply: the product is zero or not finite");
    out->D = K;
    out->tau = 0.0;
    out->e_valid = false;
    return disc;
}

namespace {

// Trapezoid step with b = (I - h (H - s)) psi formed as an MPS (Appendix B).
void trap_step_mps_rhs(ite_mps* psi, const ite_mpo* H, double h, const ite_step_opts& o, ite_step_report* rep) {
    ite_ctx* c = psi->ctx;
    const double s = step_shift(psi, H, o);
    std::vector<std::vector<double>> T;
    std::vector<int> wo;
    direct_sum_identity(H, -h, 1.0 + h * s, T, wo);
    MpoPtr Ob = load_host_mpo(c, psi->d, wo, T);
    ite_mps* b = ensure_aux(psi, psi->L, psi->d);
    sync(c);
    const auto t0 = std::chrono::steady_clock::now();
    const double disc = mpo_apply_dm(psi, Ob.get(), std::min(o.chi_max, psi->chi_max), o.cutoff, o.tie_rel, b);
    const double ms_prod = ms_since(c, t0);
    ite_step_opts ob = o;
    ob.scheme = ITE_SCHEME_BE;
    ob.shift_mode = ITE_SHIFT_FIXED;
    ob.shift = s;
    ob.rhs_mode = ITE_RHS_PROJECT;
    ite_step_report r{};
    imag_step_sweep(b, H, h, ob, &r);
    // psi <- x (same capacities: same L, d and chi_max)
    std::swap(psi->A, b->A);
    std::swap(psi->D, b->D);
    psi->tau += 2.0 * h;
    psi->energy = r.energy;
    psi->e_valid = true;
    r.tau = psi->tau;
    r.dtau = 2.0 * h;
    r.h = h;
    r.shift = s;
    r.rhs_disc = disc;
    r.aux_max_chi = 0;
    // the density-matrix product is the step's right-hand side
    r.ms_rhs += ms_prod;
    r.ms_total += ms_prod;
    if (rep) *rep = r;
}

}  // namespace

bool step_is_composite(const ite_step_opts& o) {
    return o.scheme == ITE_SCHEME_GL || (o.scheme == ITE_SCHEME_TRAP && o.rhs_mode == ITE_RHS_MPS);
}

void imag_step(ite_mps* psi, const ite_mpo* H, double h, const ite_step_opts& o, ite_step_report* rep) {
    check_step(psi, H, h, o);
    if (o.scheme == ITE_SCHEME_GL) gl_panel(psi, H, h, o, rep);
    else if (o.scheme == ITE_SCHEME_TRAP && o.rhs_mode == ITE_RHS_MPS) trap_step_mps_rhs(psi, H, h, o, rep);
    else imag_step_sweep(psi, H, h, o, rep);
}

}  // namespace ite
