// The implicit step of the MPS imaginary-time evolution, driven from the host.
//
// One step (Method, Eq. 4 and the two operations listed after it;
// Appendix B; Appendix D):
//   x <- copy of psi (normalised, right-orthonormal, centre on site 1);
//   right environments of <x|H|x>; while x = psi the mixed <x|H|psi> and
//   <x|psi> environments equal <x|H|x> and the identity;
//   left-to-right, then right-to-left over the blocks (j, j+1):
//     theta_psi = psi_j psi_(j+1);
//     b = P^T psi (backward Euler) or (1 + h s) P^T psi - h P^T H psi
//       (trapezoid): the right-hand side projected into x's basis through the
//       mixed environments;
//     GMRES on (1 - h s) v + h H_eff v = b from x_j x_(j+1);
//     SVD split (one-sided Jacobi) with truncation, environment updates;
//   normalise, energy <x|H|x>, psi <- x.
#include "engine.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <numeric>
#include <tuple>

namespace ite {

// ---------------------------------------------------------------------------
// Memory
// ---------------------------------------------------------------------------

void* dev_alloc(ite_ctx* c, size_t bytes) {
    if (bytes == 0) bytes = 16;
    bytes = (bytes + 255) & ~size_t(255);
    void* p = nullptr;
    if (c->has_alloc) {
        p = c->alloc.alloc(bytes, c->alloc.user);
        if (!p) ITE_FAIL(ITE_ENOMEM, "allocator returned NULL for " + std::to_string(bytes) + " bytes");
    } else {
        hipError_t e = hipMalloc(&p, bytes);
        if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
            ITE_FAIL(ITE_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
        HIP_CHECK(e);
    }
    return p;
}

void dev_free(ite_ctx* c, void* p) {
    if (!p) return;
    if (c->has_alloc) c->alloc.free(p, c->alloc.user);
    else (void)hipFree(p);
}

void* slot(ite_ctx* c, SlotId s, size_t bytes) {
    if (c->slot_bytes[s] < bytes) {
        if (c->slot_ptr[s]) {
            // the old buffer may still be read by queued work
            HIP_CHECK(hipStreamSynchronize(c->stream));
            dev_free(c, c->slot_ptr[s]);
            c->slot_ptr[s] = nullptr;
            c->slot_bytes[s] = 0;
        }
        const size_t nb = bytes + bytes / 8 + 256;
        c->slot_ptr[s] = dev_alloc(c, nb);
        c->slot_bytes[s] = nb;
    }
    return c->slot_ptr[s];
}

double* pinned(ite_ctx* c, size_t doubles) {
    const size_t bytes = std::max<size_t>(doubles, 64) * sizeof(double);
    if (c->pinned_bytes < bytes) {
        if (c->pinned) {
            HIP_CHECK(hipStreamSynchronize(c->stream));
            (void)hipHostFree(c->pinned);
            c->pinned = nullptr;
        }
        void* p = nullptr;
        HIP_CHECK(hipHostMalloc(&p, bytes, hipHostMallocDefault));
        c->pinned = static_cast<double*>(p);
        c->pinned_bytes = bytes;
    }
    return c->pinned;
}

void sync(ite_ctx* c) { HIP_CHECK(hipStreamSynchronize(c->stream)); }

void d2h(ite_ctx* c, double* host, const double* dev, size_t n) {
    HIP_CHECK(hipMemcpyAsync(host, dev, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
}
void h2d(ite_ctx* c, void* dev, const void* host, size_t bytes) {
    HIP_CHECK(hipMemcpyAsync(dev, host, bytes, hipMemcpyHostToDevice, c->stream));
}
// Blocking copies through the context's stream (not the legacy stream, whose
// implicit synchronisation can break a graph capture running on another
// thread's stream).
void h2d_wait(ite_ctx* c, void* dev, const void* host, size_t bytes) {
    if (!bytes) return;
    HIP_CHECK(hipMemcpyAsync(dev, host, bytes, hipMemcpyHostToDevice, c->stream));
    HIP_CHECK(hipStreamSynchronize(c->stream));
}
void d2h_wait(ite_ctx* c, void* host, const void* dev, size_t bytes) {
    if (!bytes) return;
    HIP_CHECK(hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, c->stream));
    HIP_CHECK(hipStreamSynchronize(c->stream));
}
void d2d(ite_ctx* c, double* dst, const double* src, size_t n) {
    if (n) HIP_CHECK(hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
}

// ---------------------------------------------------------------------------
// Contractions
// ---------------------------------------------------------------------------

static hipEvent_t prof_event(ite_ctx* c) {
    if (c->prof_used == c->prof_events.size()) {
        hipEvent_t e;
        HIP_CHECK(hipEventCreate(&e));
        c->prof_events.push_back(e);
    }
    return c->prof_events[c->prof_used++];
}

// Fold the recorded launch spans into the totals (synchronises the stream).
void prof_collect(ite_ctx* c) {
    if (c->prof_kind.empty()) return;
    HIP_CHECK(hipStreamSynchronize(c->stream));
    for (size_t i = 0; i < c->prof_kind.size(); ++i) {
        float ms = 0.f;
        HIP_CHECK(hipEventElapsedTime(&ms, c->prof_events[2 * i], c->prof_events[2 * i + 1]));
        c->prof_ms[c->prof_kind[i]] += ms;
        c->prof_timed[c->prof_kind[i]]++;
    }
    c->prof_kind.clear();
    c->prof_used = 0;
}

namespace {

// The context's LaunchProbe: counts launches, times every launch of an FP64
// GEMM and every jac_period-th launch of each Jacobi kernel.
struct CtxProbe final : LaunchProbe {
    ite_ctx* c;
    explicit CtxProbe(ite_ctx* cc) : c(cc) {}
    bool begin(int kind, hipStream_t s) override {
        const long long n = c->prof_launches[kind]++;
        if (kind != PK_GEMM && n % c->jac_period != 0) return false;
        if (c->prof_kind.size() >= 4096) prof_collect(c);
        HIP_CHECK(hipEventRecord(prof_event(c), s));
        return true;
    }
    void end(int kind, hipStream_t s) override {
        HIP_CHECK(hipEventRecord(prof_event(c), s));
        c->prof_kind.push_back(kind);
    }
    void work(int kind, double flops, double bytes) override {
        c->prof_flops[kind] += flops;
        c->prof_bytes[kind] += bytes;
    }
};

}  // namespace

// Concurrent workgroups of the GEMM kernels on the context's device (two per
// compute unit).
static int gemm_slots(ite_ctx* c) {
    if (c->gemm_slots == 0) {
        int cus = 0;
        HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device));
        c->gemm_slots = 2 * std::max(cus, 1);
    }
    return c->gemm_slots;
}

void gemm(ite_ctx* c, bool tA, bool tB, int M, int N, int K, double alpha, const double* A, long lda,
          const double* B, long ldb, double beta, const double* C, long ldc, double* D, long ldd) {
    Gemm g;
    g.M = M; g.N = N; g.K = K; g.tA = tA; g.tB = tB;
    g.alpha = alpha; g.beta = beta;
    g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.C = C; g.ldc = ldc; g.D = D; g.ldd = ldd;
    // an output too small to fill the chip's workgroup slots but with a long
    // K: K parts as one batch, summed in a fixed order
    const int parts = M > 0 && N > 0 ? splitk_parts(M, N, K, gemm_slots(c)) : 1;
    double* work = parts > 1 ? slot_t<double>(c, SL_SPLITK, (size_t)parts * M * N) : nullptr;
    if (c->prof_on && M > 0 && N > 0) {
        CtxProbe pr(c);
        pr.begin(PK_GEMM, c->stream);
        gemm_f64_splitk(g, parts, work, c->stream);
        pr.end(PK_GEMM, c->stream);
        pr.work(PK_GEMM, 2.0 * M * N * (double)K,
                8.0 * ((double)M * K + (double)K * N + (C && beta != 0.0 ? 2.0 : 1.0) * (double)M * N));
        return;
    }
    gemm_f64_splitk(g, parts, work, c->stream);
}

void stage(ite_ctx* c, const CsrDev& m, Stage st) {
    st.I = m.I;
    st.O = m.O;
    st.rowptr = m.rowptr;
    st.col = m.col;
    st.val = m.val;
    st.nnz = m.nnz;
    stage_f64(st, c->stream);
}

void two_site(ite_ctx* c, int Dl, int d1, int Dm, int d2, int Dr, const double* A1, const double* A2,
              double* theta) {
    gemm(c, false, false, Dl * d1, d2 * Dr, Dm, 1.0, A1, Dm, A2, (long)d2 * Dr, 0.0, nullptr, 0, theta,
         (long)d2 * Dr);
}

// H_eff theta in three stages (Appendix B's local problem):
//   X1[(a' w), (s t c)]   = L[(a' w), a] theta[a, (s t c)]           GEMM
//   X3[a'][(p q u)][c]    = WW[(p q u), (w s t)] X1[a'][(w s t)][c]  sparse MPO stage
//   y[(a' p q), c']       = X3[(a' p q), (u c)] R[c', (u c)]^T        GEMM (+ alpha Cadd)
static size_t lo_bytes(Prec p) { return p == Prec::F32 ? 4 : 2; }

// Round n FP64 values to the operand precision into dst.
static void to_lo(ite_ctx* c, Prec p, const double* x, void* dst, size_t n) {
    if (p == Prec::F32) convert_f32(x, static_cast<float*>(dst), n, c->stream);
    else convert_bf16(x, static_cast<uint16_t*>(dst), n, c->stream);
}

static void gemm_lo(ite_ctx* c, Prec p, bool tA, bool tB, int M, int N, int K, double alpha, const void* A,
                    long lda, const void* B, long ldb, double beta, const double* C, long ldc, double* D, long ldd,
                    float* Df = nullptr) {
    Gemm g;
    g.M = M; g.N = N; g.K = K; g.tA = tA; g.tB = tB;
    g.alpha = alpha; g.beta = beta;
    g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.C = C; g.ldc = ldc; g.D = D; g.ldd = ldd;
    g.Df = Df;
    if (p == Prec::F32) {
        // an FP64 output too small to fill the chip with a long K: K parts,
        // as for the FP64 products
        const int parts = !Df && M > 0 && N > 0 ? splitk_parts(M, N, K, gemm_slots(c)) : 1;
        if (parts > 1) gemm_f32_splitk(g, parts, slot_t<double>(c, SL_SPLITK, (size_t)parts * M * N), c->stream);
        else gemm_f32(g, c->stream);
    } else {
        gemm_bf16(g, c->stream);
    }
}

void lo_shadows(ite_ctx* c, const HeffShape& s, Prec prec, const double* L, const double* R, const void** Llo,
                const void** Rlo) {
    const size_t eb = lo_bytes(prec);
    const size_t nl = (size_t)s.Dxl * s.w0 * s.Dyl, nr = (size_t)s.Dxr * s.w2 * s.Dyr;
    void* l = slot(c, SL_LO_L, nl * eb);
    void* r = slot(c, SL_LO_R, nr * eb);
    to_lo(c, prec, L, l, nl);
    to_lo(c, prec, R, r, nr);
    *Llo = l;
    *Rlo = r;
}

void heff_apply(ite_ctx* c, const HeffShape& s, const double* L, const CsrDev& ww, const double* R,
                const double* theta, double beta, double alpha, const double* Cadd, double* y, Prec prec,
                const void* Llo, const void* Rlo) {
    const int I = s.w0 * s.d1 * s.d2, O = s.d1 * s.d2 * s.w2;
    const size_t nx = (size_t)s.Dxl * std::max(I, O) * s.Dyr;
    if (prec != Prec::F64) {
        // operands rounded to FP32 / BF16, FP32 accumulation in the matrix
        // cores; the first intermediate in FP32 (the accumulator's precision,
        // half the traffic of FP64), the second in the operand precision, the
        // output in FP64
        const size_t eb = lo_bytes(prec);
        if (!Llo || !Rlo) lo_shadows(c, s, prec, L, R, &Llo, &Rlo);
        const size_t nth = (size_t)s.Dyl * s.d1 * s.d2 * s.Dyr;
        void* tlo = slot(c, SL_LO_T, nth * eb);
        void* x3lo = slot(c, SL_LO_X, nx * eb);
        float* X1 = static_cast<float*>(slot(c, SL_X1, nx * sizeof(float)));
        to_lo(c, prec, theta, tlo, nth);
        gemm_lo(c, prec, false, false, s.Dxl * s.w0, s.d1 * s.d2 * s.Dyr, s.Dyl, 1.0, Llo, s.Dyl, tlo,
                (long)s.d1 * s.d2 * s.Dyr, 0.0, nullptr, 0, nullptr, (long)s.d1 * s.d2 * s.Dyr, X1);
        Stage st;
        st.G = s.Dxl; st.C = s.Dyr;
        st.in_f32 = X1; st.in_gs = (long)I * s.Dyr; st.in_s1 = s.Dyr;
        st.out_gs = (long)O * s.Dyr; st.out_s1 = s.Dyr;
        st.out_prec = prec == Prec::F32 ? 1 : 2;
        st.out_lo = x3lo;
        stage(c, ww, st);
        gemm_lo(c, prec, false, true, s.Dxl * s.d1 * s.d2, s.Dxr, s.w2 * s.Dyr, beta, x3lo, (long)s.w2 * s.Dyr,
                Rlo, (long)s.w2 * s.Dyr, alpha, Cadd, s.Dxr, y, s.Dxr);
        return;
    }
    double* X1 = slot_t<double>(c, SL_X1, nx);
    double* X3 = slot_t<double>(c, SL_X3, nx);
    gemm(c, false, false, s.Dxl * s.w0, s.d1 * s.d2 * s.Dyr, s.Dyl, 1.0, L, s.Dyl, theta,
         (long)s.d1 * s.d2 * s.Dyr, 0.0, nullptr, 0, X1, (long)s.d1 * s.d2 * s.Dyr);
    Stage st;
    st.G = s.Dxl; st.C = s.Dyr;
    st.in = X1; st.in_gs = (long)I * s.Dyr; st.in_s1 = s.Dyr;
    st.out = X3; st.out_gs = (long)O * s.Dyr; st.out_s1 = s.Dyr;
    stage(c, ww, st);
    gemm(c, false, true, s.Dxl * s.d1 * s.d2, s.Dxr, s.w2 * s.Dyr, beta, X3, (long)s.w2 * s.Dyr, R,
         (long)s.w2 * s.Dyr, alpha, Cadd, s.Dxr, y, s.Dxr);
}

void overlap_apply(ite_ctx* c, int Dxl, int Dyl, int Dxr, int Dyr, int d1, int d2, const double* Lo,
                   const double* Ro, const double* theta, double alpha, double* y) {
    const long nmid = (long)d1 * d2;
    const double* T = theta;
    if (Lo) {
        double* X1 = slot_t<double>(c, SL_X1, (size_t)Dxl * nmid * Dyr);
        gemm(c, false, false, Dxl, (int)(nmid * Dyr), Dyl, Ro ? 1.0 : alpha, Lo, Dyl, theta, nmid * Dyr, 0.0,
             nullptr, 0, X1, nmid * Dyr);
        T = X1;
        if (!Ro) {
            d2d(c, y, X1, (size_t)Dxl * nmid * Dyr);
            return;
        }
    }
    if (Ro) {
        gemm(c, false, true, (int)(Dxl * nmid), Dxr, Dyr, alpha, T, Dyr, Ro, Dyr, 0.0, nullptr, 0, y, Dxr);
        return;
    }
    axpby((size_t)Dxl * nmid * Dyr, alpha, theta, 0.0, nullptr, y, c->stream);
}

void env_left(ite_ctx* c, int Dxa, int Dya, int Dxb, int Dyb, int d, int wl, int wr, const double* E,
              const double* X, const CsrDev* W, const double* Y, double* Eout) {
    if (W) {
        double* T1 = slot_t<double>(c, SL_X1, (size_t)Dxa * wl * d * Dyb);
        double* T2 = slot_t<double>(c, SL_X3, (size_t)Dxa * d * wr * Dyb);
        // T1[(a' w), (s b)] = E[(a' w), a] Y[a, (s b)]
        gemm(c, false, false, Dxa * wl, d * Dyb, Dya, 1.0, E, Dya, Y, (long)d * Dyb, 0.0, nullptr, 0, T1,
             (long)d * Dyb);
        // T2[a'][(p v)][b] = WL[(p v), (w s)] T1[a'][(w s)][b]
        Stage st;
        st.G = Dxa; st.C = Dyb;
        st.in = T1; st.in_gs = (long)wl * d * Dyb; st.in_s1 = Dyb;
        st.out = T2; st.out_gs = (long)d * wr * Dyb; st.out_s1 = Dyb;
        stage(c, *W, st);
        // E'[b', (v b)] = X[(a' p), b']^T T2[(a' p), (v b)]
        gemm(c, true, false, Dxb, wr * Dyb, Dxa * d, 1.0, X, Dxb, T2, (long)wr * Dyb, 0.0, nullptr, 0, Eout,
             (long)wr * Dyb);
    } else {
        double* T1 = slot_t<double>(c, SL_X1, (size_t)Dxa * d * Dyb);
        gemm(c, false, false, Dxa, d * Dyb, Dya, 1.0, E, Dya, Y, (long)d * Dyb, 0.0, nullptr, 0, T1,
             (long)d * Dyb);
        gemm(c, true, false, Dxb, Dyb, Dxa * d, 1.0, X, Dxb, T1, Dyb, 0.0, nullptr, 0, Eout, Dyb);
    }
}

void env_right(ite_ctx* c, int Dxa, int Dya, int Dxb, int Dyb, int d, int wl, int wr, const double* E,
               const double* X, const CsrDev* W, const double* Y, double* Eout) {
    const int we = W ? wr : 1;
    double* T1 = slot_t<double>(c, SL_X1, (size_t)Dxa * we * Dyb * d);
    double* T2 = slot_t<double>(c, SL_X3, (size_t)d * Dxa * (W ? wl : 1) * Dyb);
    // T1[(c' v), (b s)] = E[(c' v), c] Y[(b s), c]^T
    gemm(c, false, true, Dxa * we, Dyb * d, Dya, 1.0, E, Dya, Y, Dya, 0.0, nullptr, 0, T1, (long)Dyb * d);
    Stage st;
    st.G = Dxa; st.C = Dyb;
    st.in = T1; st.in_gs = (long)we * Dyb * d; st.in_div = d; st.in_s1 = (long)Dyb * d; st.in_s2 = 1;
    st.in_cs = d;
    st.out = T2;
    if (W) {
        // T2[p][c'][w][b] = WR[(p w), (v s)] T1[c'][v][b][s]
        st.out_gs = (long)wl * Dyb; st.out_div = wl; st.out_s1 = (long)Dxa * wl * Dyb; st.out_s2 = Dyb;
        stage(c, *W, st);
        gemm(c, false, false, Dxb, wl * Dyb, d * Dxa, 1.0, X, (long)d * Dxa, T2, (long)wl * Dyb, 0.0, nullptr,
             0, Eout, (long)wl * Dyb);
    } else {
        ITE_FAIL(ITE_EINVAL, "env_right overlap needs the identity stage");
    }
}

void env_right_overlap_pub(ite_ctx* c, const CsrDev& ident, int Dxa, int Dya, int Dxb, int Dyb, int d,
                              const double* E, const double* X, const double* Y, double* Eout) {
    double* T1 = slot_t<double>(c, SL_X1, (size_t)Dxa * Dyb * d);
    double* T2 = slot_t<double>(c, SL_X3, (size_t)d * Dxa * Dyb);
    // T1[c', (b s)] = E[c', c] Y[(b s), c]^T
    gemm(c, false, true, Dxa, Dyb * d, Dya, 1.0, E, Dya, Y, Dya, 0.0, nullptr, 0, T1, (long)Dyb * d);
    // T2[s][c'][b] = T1[c'][b][s]
    Stage st;
    st.G = Dxa; st.C = Dyb;
    st.in = T1; st.in_gs = (long)Dyb * d; st.in_s1 = 1; st.in_cs = d;
    st.out = T2; st.out_gs = Dyb; st.out_s1 = (long)Dxa * Dyb;
    stage(c, ident, st);
    // E'[b', b] = X[b', (s c')] T2[(s c'), b]
    gemm(c, false, false, Dxb, Dyb, d * Dxa, 1.0, X, (long)d * Dxa, T2, Dyb, 0.0, nullptr, 0, Eout, Dyb);
}

double dot(ite_ctx* c, const double* x, const double* y, size_t n) {
    const int nb = reduce_blocks(n);
    double* part = slot_t<double>(c, SL_PART, (size_t)nb * 64 + 64);
    double* sm = slot_t<double>(c, SL_SMALL, 512);
    dot_partials(x, y, n, part, c->stream);
    finish_partials(part, 1, nb, sm + 256, 0, c->stream);
    double* h = pinned(c, 64);
    d2h(c, h, sm + 256, 1);
    sync(c);
    return h[0];
}

// ---------------------------------------------------------------------------
// Truncated split by one-sided Jacobi
// ---------------------------------------------------------------------------

int truncation_rank(const std::vector<double>& s, double cutoff, int chi_max, double tie_rel) {
    const int r = (int)s.size();
    if (r == 0) return 0;
    double total = 0.0;
    for (double v : s) total += v * v;
    int k = r;
    if (cutoff > 0.0 && total > 0.0) {
        // tail[k] = sum_{i >= k} s_i^2, accumulated from the smallest value up
        std::vector<double> tail(r + 1, 0.0);
        for (int i = r - 1; i >= 0; --i) tail[i] = tail[i + 1] + s[i] * s[i];
        k = r;
        for (int kk = 1; kk <= r; ++kk)
            if (tail[kk] <= cutoff * total) { k = kk; break; }
    }
    k = std::max(1, std::min(k, chi_max));
    const double tie = tie_rel * s[0];
    while (k > 1 && k < r && s[k - 1] > tie && s[k - 1] - s[k] <= tie) --k;
    return k;
}

SplitResult split(ite_ctx* c, int dir, int Dl, int d1, int d2, int Dr, const double* theta, int chi_max,
                  double cutoff, double tie_rel, double* A1, double* A2, std::vector<double>* sigma) {
    const int m = Dl * d1, n = d2 * Dr;
    const int p = dir == 0 ? m : n, q = dir == 0 ? n : m, ld = p + q;
    double* Z = slot_t<double>(c, SL_Z, (size_t)p * ld);
    size_t ngram = 0, nrot = 0, noff = 0;
    jacobi_workspace(p, q, &ngram, &nrot, &noff);
    double* gram = slot_t<double>(c, SL_GRAM, ngram);
    double* rot = slot_t<double>(c, SL_ROT, nrot);
    double* off = slot_t<double>(c, SL_OFF, noff);
    double* norms = slot_t<double>(c, SL_NORM, (size_t)p + 16);
    int* perm = slot_t<int>(c, SL_PERM, (size_t)p + 16);
    jacobi_input(theta, m, n, dir, Z, c->stream);
    // Householder preconditioning: the Jacobi then works on the rows of R,
    // of which only the first min(p, q) can be non-zero
    int pj = p;
    if (householder_applies(p, q)) {
        double* qws = slot_t<double>(c, SL_QR, householder_workspace(p, q, ld));
        householder_rows(Z, p, q, ld, qws, c->stream);
        pj = std::min(p, q);
    }
    double* host = pinned(c, (size_t)p + 64);
    const double tol = 8.0 * std::sqrt((double)std::max(q, 1)) * 2.220446049250313e-16;
    CtxProbe probe(c);
    JacobiResult jr = jacobi_rows(Z, pj, q, ld, tol, 60, gram, rot, off, host, c->stream,
                                  c->prof_on ? &probe : nullptr);
    row_norms(Z, p, q, ld, norms, c->stream);
    d2h(c, host, norms, p);
    sync(c);
    std::vector<int> idx(p);
    std::iota(idx.begin(), idx.end(), 0);
    std::vector<double> nv(host, host + p);
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return nv[a] > nv[b]; });
    const int r = std::min(m, n);
    std::vector<double> s(r);
    for (int i = 0; i < r; ++i) s[i] = nv[idx[i]];
    SplitResult res;
    res.k = truncation_rank(s, cutoff, chi_max, tie_rel);
    double total = 0.0, kept = 0.0;
    for (int i = 0; i < r; ++i) total += s[i] * s[i];
    for (int i = res.k; i < r; ++i) kept += s[i] * s[i];
    res.disc = total > 0.0 ? kept / total : 0.0;
    res.sweeps = jr.sweeps;
    if (sigma) *sigma = s;
    int* hp = reinterpret_cast<int*>(host);
    std::memcpy(hp, idx.data(), sizeof(int) * res.k);
    h2d(c, perm, hp, sizeof(int) * res.k);
    if (dir == 0) gather_split(Z, ld, perm, res.k, 0, q, A2, q, p, A1, c->stream);
    else gather_split(Z, ld, perm, res.k, q, p, A2, 0, q, A1, c->stream);
    sync(c);   // the pinned staging buffer is reused by the next call
    return res;
}

// ---------------------------------------------------------------------------
// GMRES local solve
// ---------------------------------------------------------------------------

// SolveStats of a device record (see hess_solve): [0] residual, [1] products,
// [2] flags, [4] the residual products among them.  low: every product with
// low-precision operands; mixed: the residual products FP64, the others low.
static SolveStats stats_from(const double* rec, bool low, bool mixed = false) {
    SolveStats st;
    st.res_rel = rec[0];
    if (mixed) {
        st.matvecs64 = (int)rec[4];
        st.matvecs_lo = (int)rec[1] - (int)rec[4];
    } else {
        (low ? st.matvecs_lo : st.matvecs64) = (int)rec[1];
    }
    st.flags = (int)rec[2];
    return st;
}

static void op_apply(ite_ctx* c, const LocalOp& op, const double* v, double* y) {
    heff_apply(c, op.s, op.L, *op.ww, op.R, v, op.beta, op.alpha, v, y, op.prec, op.Llo, op.Rlo);
}

// GMRES(m) with the fixed budget (no tolerance: m Arnoldi steps per cycle,
// fewer only at an invariant subspace), entirely on the device: the Arnoldi
// steps, then the cycle's least-squares problem (Givens rotations, the
// breakdown test, back substitution: hess_solve) and x += V y, with no wait
// for the host.  The residual estimate, the product count and the flags are
// accumulated in the device record `stats` (8 doubles); when it is null a
// context slot is used and read back once at the end.  Steps after a
// breakdown (the next basis vector divides by a vanishing norm) are computed
// and discarded; the counts report the products whose results enter the
// solution.  Same kernels in the same order as the tolerance-driven loop
// below.
static SolveStats gmres_budget(ite_ctx* c, const LocalOp& op, const double* b, double* x, int m, int max_cycles,
                               bool x_is_zero, double* stats = nullptr) {
    const size_t n = op.n();
    const int mm = (int)std::min<size_t>((size_t)m, n);
    constexpr int HC = HESS_HC;   // per column: [0,64) first-pass coefficients, [64,128) second pass, 128 norm
    double* V = slot_t<double>(c, SL_V, (size_t)(mm + 1) * n);
    double* w = slot_t<double>(c, SL_W, n);
    const int nb = reduce_blocks(n);
    double* part = slot_t<double>(c, SL_PART, (size_t)nb * 64 + 64);
    double* hd = slot_t<double>(c, SL_HESS, (size_t)mm * HC + 8 + 64 + 8);
    double* bnorm_d = hd + (size_t)mm * HC;       // ||b||
    double* beta_d = bnorm_d + 1;                 // ||r0||
    double* ydev = hd + (size_t)mm * HC + 8;      // combination coefficients (64)
    const bool own_stats = stats == nullptr;
    if (own_stats) stats = hd + (size_t)mm * HC + 8 + 64;
    fill(stats, 0.0, 8, c->stream);
    dot_partials(b, b, n, part, c->stream);
    finish_partials(part, 1, nb, bnorm_d, 2, c->stream);
    for (int cyc = 0; cyc < max_cycles; ++cyc) {
        // r0 = b - A x
        bool r_product = false;
        if (x_is_zero && cyc == 0) {
            d2d(c, V, b, n);
        } else {
            op_apply(c, op, x, V);
            r_product = true;
            axpby(n, 1.0, b, -1.0, V, V, c->stream);
        }
        dot_partials(V, V, n, part, c->stream);
        finish_partials(part, 1, nb, beta_d, 2, c->stream);
        scale_inv(V, beta_d, V, n, c->stream);
        for (int k = 0; k < mm; ++k) {
            double* col = hd + (size_t)k * HC;
            double* vnext = k + 1 < mm ? V + (size_t)(k + 1) * n : nullptr;
            op_apply(c, op, V + (size_t)k * n, w);
            if (cgs2_small(V, (long)n, k + 1, w, n, col, vnext, c->stream)) continue;
            mdot_partials(V, (long)n, k + 1, w, n, part, c->stream);
            finish_partials(part, k + 1, nb, col, 0, c->stream);
            gemv_sub(V, (long)n, k + 1, col, w, n, c->stream);
            mdot_partials(V, (long)n, k + 1, w, n, part, c->stream);
            finish_partials(part, k + 1, nb, col + 64, 0, c->stream);
            gemv_sub(V, (long)n, k + 1, col + 64, w, n, c->stream);
            dot_partials(w, w, n, part, c->stream);
            finish_partials(part, 1, nb, col + 128, 2, c->stream);
            if (vnext) scale_inv(w, col + 128, vnext, n, c->stream);
        }
        hess_solve(hd, mm, ydev, stats, r_product, cyc + 1 == max_cycles, c->stream);
        gemv_add(V, (long)n, mm, ydev, x, n, c->stream);
    }
    SolveStats st;
    if (own_stats) {
        double* host = pinned(c, 64);
        d2h(c, host, stats, 4);
        sync(c);
        st = stats_from(host, op.prec != Prec::F64);
    }
    return st;
}

// GMRES(m) (Saad and Schultz) with classical Gram-Schmidt applied twice; the
// Hessenberg column comes to the host once per Arnoldi step, where Givens
// rotations keep the least-squares residual.  Vectors, Gram-Schmidt and the
// Hessenberg problem are FP64 whatever the precision of the products.  With
// x_is_zero the first residual is b itself (no product).
static SolveStats gmres(ite_ctx* c, const LocalOp& op, const double* b, double* x, int m, int max_cycles,
                        double tol, bool x_is_zero = false) {
    if (tol <= 0) return gmres_budget(c, op, b, x, m, max_cycles, x_is_zero);
    SolveStats st;
    const bool lo = op.prec != Prec::F64;
    int& mv = lo ? st.matvecs_lo : st.matvecs64;
    const size_t n = op.n();
    const int mm = (int)std::min<size_t>((size_t)m, n);
    double* V = slot_t<double>(c, SL_V, (size_t)(mm + 1) * n);
    double* w = slot_t<double>(c, SL_W, n);
    const int nb = reduce_blocks(n);
    double* part = slot_t<double>(c, SL_PART, (size_t)nb * 64 + 64);
    double* sm = slot_t<double>(c, SL_SMALL, 512);   // [0,64) h1, [64,128) h2, 128 norm, [192,256) y
    double* host = pinned(c, 512);
    const double bnorm = std::sqrt(std::max(0.0, dot(c, b, b, n)));
    std::vector<double> H((size_t)(mm + 1) * mm), cs(mm), sn(mm), g(mm + 1), y(mm);
    for (int cyc = 0; cyc < max_cycles; ++cyc) {
        // r0 = b - A x
        if (x_is_zero && cyc == 0) {
            d2d(c, V, b, n);
        } else {
            op_apply(c, op, x, V);
            mv++;
            axpby(n, 1.0, b, -1.0, V, V, c->stream);
        }
        dot_partials(V, V, n, part, c->stream);
        finish_partials(part, 1, nb, sm + 128, 2, c->stream);
        d2h(c, host, sm + 128, 1);
        sync(c);
        const double beta = host[0];
        st.res_rel = bnorm > 0 ? beta / bnorm : 0.0;
        if (!(beta > 0.0) || (tol > 0 && beta <= tol * bnorm)) return st;
        scale_inv(V, sm + 128, V, n, c->stream);
        std::fill(H.begin(), H.end(), 0.0);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int kused = 0;
        bool converged = false;
        for (int k = 0; k < mm; ++k) {
            op_apply(c, op, V + (size_t)k * n, w);
            mv++;
            if (!cgs2_small(V, (long)n, k + 1, w, n, sm, nullptr, c->stream)) {
                mdot_partials(V, (long)n, k + 1, w, n, part, c->stream);
                finish_partials(part, k + 1, nb, sm, 0, c->stream);
                gemv_sub(V, (long)n, k + 1, sm, w, n, c->stream);
                mdot_partials(V, (long)n, k + 1, w, n, part, c->stream);
                finish_partials(part, k + 1, nb, sm + 64, 0, c->stream);
                gemv_sub(V, (long)n, k + 1, sm + 64, w, n, c->stream);
                dot_partials(w, w, n, part, c->stream);
                finish_partials(part, 1, nb, sm + 128, 2, c->stream);
            }
            d2h(c, host, sm, 129);
            sync(c);
            for (int i = 0; i <= k; ++i) H[(size_t)i * mm + k] = host[i] + host[64 + i];
            const double hnext = host[128];
            // apply the previous rotations to column k
            for (int i = 0; i < k; ++i) {
                const double a = H[(size_t)i * mm + k], bb = H[(size_t)(i + 1) * mm + k];
                H[(size_t)i * mm + k] = cs[i] * a + sn[i] * bb;
                H[(size_t)(i + 1) * mm + k] = -sn[i] * a + cs[i] * bb;
            }
            const double a = H[(size_t)k * mm + k];
            const double rr = std::hypot(a, hnext);
            cs[k] = rr > 0 ? a / rr : 1.0;
            sn[k] = rr > 0 ? hnext / rr : 0.0;
            H[(size_t)k * mm + k] = rr;
            g[k + 1] = -sn[k] * g[k];
            g[k] = cs[k] * g[k];
            kused = k + 1;
            const double res = std::fabs(g[k + 1]);
            st.res_rel = bnorm > 0 ? res / bnorm : 0.0;
            if (hnext <= 1e-14 * beta) {
                st.flags |= ITE_FLAG_BREAKDOWN;
                converged = true;
                break;
            }
            if (tol > 0 && res <= tol * bnorm) {
                converged = true;
                break;
            }
            scale_inv(w, sm + 128, V + (size_t)(k + 1) * n, n, c->stream);
        }
        // back substitution R y = g
        for (int i = kused - 1; i >= 0; --i) {
            double s = g[i];
            for (int j = i + 1; j < kused; ++j) s -= H[(size_t)i * mm + j] * y[j];
            const double dgn = H[(size_t)i * mm + i];
            y[i] = dgn != 0.0 ? s / dgn : 0.0;
        }
        for (int i = 0; i < kused; ++i) host[256 + i] = y[i];
        h2d(c, sm + 192, host + 256, sizeof(double) * kused);
        gemv_add(V, (long)n, kused, sm + 192, x, n, c->stream);
        sync(c);
        if (converged) return st;
        if (tol <= 0) {
            if (cyc + 1 == max_cycles) st.flags |= ITE_FLAG_BUDGET_EXHAUSTED;
            continue;
        }
        if (cyc + 1 == max_cycles) st.flags |= ITE_FLAG_BUDGET_EXHAUSTED;
    }
    return st;
}

// Local solve.  FP64: GMRES on the FP64 operator.  FP32_IR / BF16_IR: mixed
// precision iterative refinement -- the residual r = b - A x is formed with
// the FP64 operator, the correction solves A d = r by GMRES whose products use
// FP32 or BF16 operands with FP32 accumulation, then x += d; max_refine
// corrections, stopping early once ||r|| <= tol_refine ||b||.  With a
// residual target the reported residual is the last FP64 one; without one
// (tol_refine = 0: a fixed number of corrections, the analogue of the fixed
// GMRES budget) the residual after the last correction is not formed and the
// inner GMRES estimate, scaled by ||r|| / ||b||, is reported instead.
SolveStats local_solve(ite_ctx* c, const LocalOp& op, const double* b, double* x, int m, int max_cycles,
                       double tol, int precision, int max_refine, double tol_refine, double* stats_dev) {
    if (precision == ITE_PREC_FP64 && tol <= 0 && stats_dev) {
        gmres_budget(c, op, b, x, m, max_cycles, false, stats_dev);
        SolveStats st;
        st.deferred = true;
        return st;
    }
    if (precision == ITE_PREC_FP64) return gmres(c, op, b, x, m, max_cycles, tol);
    const Prec p = precision == ITE_PREC_FP32_IR ? Prec::F32 : Prec::BF16;
    const size_t n = op.n();
    const size_t eb = lo_bytes(p);
    const size_t nl = (size_t)op.s.Dxl * op.s.w0 * op.s.Dyl, nr = (size_t)op.s.Dxr * op.s.w2 * op.s.Dyr;
    void* Llo = slot(c, SL_LO_L, nl * eb);
    void* Rlo = slot(c, SL_LO_R, nr * eb);
    to_lo(c, p, op.L, Llo, nl);
    to_lo(c, p, op.R, Rlo, nr);
    LocalOp lop = op;
    lop.prec = p;
    lop.Llo = Llo;
    lop.Rlo = Rlo;
    double* r = slot_t<double>(c, SL_R64, n);
    double* d = slot_t<double>(c, SL_D64, n);
    const double bnorm = std::sqrt(std::max(0.0, dot(c, b, b, n)));
    SolveStats st;
    for (int it = 0;; ++it) {
        op_apply(c, op, x, r);
        st.matvecs64++;
        axpby(n, 1.0, b, -1.0, r, r, c->stream);
        const double rn = std::sqrt(std::max(0.0, dot(c, r, r, n)));
        st.res_rel = bnorm > 0 ? rn / bnorm : 0.0;
        if (!(rn > 0.0) || (tol_refine > 0 && rn <= tol_refine * bnorm)) break;
        if (it == max_refine) {
            st.flags |= ITE_FLAG_REFINE_LIMIT;
            break;
        }
        fill(d, 0.0, n, c->stream);
        SolveStats in = gmres(c, lop, r, d, m, max_cycles, tol, true);
        st.matvecs_lo += in.matvecs_lo;
        st.flags |= in.flags & ~ITE_FLAG_BUDGET_EXHAUSTED;
        axpby(n, 1.0, d, 1.0, x, x, c->stream);
        if (tol_refine <= 0 && it + 1 == max_refine) {
            st.res_rel = in.res_rel * st.res_rel;
            break;
        }
    }
    return st;
}

// ---------------------------------------------------------------------------
// MPO handle
// ---------------------------------------------------------------------------

CsrHost dense_to_csr(const std::vector<double>& M, int O, int I) {
    CsrHost h;
    h.I = I;
    h.O = O;
    h.rowptr.push_back(0);
    for (int o = 0; o < O; ++o) {
        for (int i = 0; i < I; ++i) {
            const double v = M[(size_t)o * I + i];
            if (v != 0.0) {
                h.col.push_back(i);
                h.val.push_back(v);
            }
        }
        h.rowptr.push_back((int)h.col.size());
    }
    return h;
}

std::vector<CsrDev> upload_csr(ite_ctx* c, const std::vector<CsrHost>& hs, void** block) {
    size_t bytes = 0;
    for (const auto& h : hs) {
        bytes += ((h.rowptr.size() * sizeof(int) + 255) & ~size_t(255));
        bytes += ((h.col.size() * sizeof(int) + 255) & ~size_t(255)) + 256;
        bytes += ((h.val.size() * sizeof(double) + 255) & ~size_t(255)) + 256;
    }
    *block = dev_alloc(c, bytes);
    std::vector<char> staging(bytes, 0);
    std::vector<CsrDev> out;
    size_t pos = 0;
    char* base = static_cast<char*>(*block);
    for (const auto& h : hs) {
        CsrDev dv;
        dv.I = h.I;
        dv.O = h.O;
        dv.nnz = (int)h.val.size();
        dv.rowptr = reinterpret_cast<int*>(base + pos);
        std::memcpy(staging.data() + pos, h.rowptr.data(), h.rowptr.size() * sizeof(int));
        pos += ((h.rowptr.size() * sizeof(int) + 255) & ~size_t(255));
        dv.col = reinterpret_cast<int*>(base + pos);
        if (!h.col.empty()) std::memcpy(staging.data() + pos, h.col.data(), h.col.size() * sizeof(int));
        pos += ((h.col.size() * sizeof(int) + 255) & ~size_t(255)) + 256;
        dv.val = reinterpret_cast<double*>(base + pos);
        if (!h.val.empty()) std::memcpy(staging.data() + pos, h.val.data(), h.val.size() * sizeof(double));
        pos += ((h.val.size() * sizeof(double) + 255) & ~size_t(255)) + 256;
        out.push_back(dv);
    }
    try {
        h2d_wait(c, *block, staging.data(), bytes);
    } catch (...) {
        dev_free(c, *block);
        *block = nullptr;
        throw;
    }
    return out;
}

ite_mpo* mpo_load(ite_ctx* c, int L, const int* d, const int* w, const double* const* W) {
    ITE_REQUIRE(L >= 2, "mpo_load: L must be >= 2");
    ITE_REQUIRE(d && w && W, "mpo_load: NULL array");
    ITE_REQUIRE(w[0] == 1 && w[L] == 1, "mpo_load: boundary MPO bond dimensions must be 1");
    for (int i = 0; i < L; ++i) {
        ITE_REQUIRE(d[i] >= 1 && d[i] <= 8, "mpo_load: local dimension must be in 1..8");
        ITE_REQUIRE(W[i] != nullptr, "mpo_load: NULL tensor");
    }
    for (int i = 0; i <= L; ++i) ITE_REQUIRE(w[i] >= 1 && w[i] <= 16, "mpo_load: MPO bond dimension must be in 1..16");
    std::unique_ptr<ite_mpo> m(new ite_mpo);
    m->ctx = c;
    m->L = L;
    m->d.assign(d, d + L);
    m->w.assign(w, w + L + 1);
    m->Wh.resize(L);
    for (int i = 0; i < L; ++i) {
        const size_t n = (size_t)w[i] * w[i + 1] * d[i] * d[i];
        m->Wh[i].assign(W[i], W[i] + n);
        for (double v : m->Wh[i]) ITE_REQUIRE(std::isfinite(v), "mpo_load: non-finite MPO entry");
    }
    auto Wat = [&](int i, int a, int b, int p, int s) {
        const int di = m->d[i];
        return m->Wh[i][(((size_t)a * m->w[i + 1] + b) * di + p) * di + s];
    };
    std::vector<CsrHost> hp, hl, hr, hi;
    for (int j = 0; j + 1 < L; ++j) {
        const int w0 = w[j], w1 = w[j + 1], w2 = w[j + 2], d1 = d[j], d2 = d[j + 1];
        const int I = w0 * d1 * d2, O = d1 * d2 * w2;
        std::vector<double> M((size_t)O * I, 0.0);
        for (int a = 0; a < w0; ++a)
            for (int s = 0; s < d1; ++s)
                for (int t = 0; t < d2; ++t)
                    for (int p = 0; p < d1; ++p)
                        for (int q = 0; q < d2; ++q)
                            for (int u = 0; u < w2; ++u) {
                                double acc = 0.0;
                                for (int v = 0; v < w1; ++v) acc += Wat(j, a, v, p, s) * Wat(j + 1, v, u, q, t);
                                M[((size_t)(p * d2 + q) * w2 + u) * I + (a * d1 + s) * d2 + t] = acc;
                            }
        hp.push_back(dense_to_csr(M, O, I));
    }
    for (int j = 0; j < L; ++j) {
        const int wl = w[j], wr = w[j + 1], dj = d[j];
        std::vector<double> ML((size_t)dj * wr * wl * dj), MR((size_t)dj * wl * wr * dj);
        for (int a = 0; a < wl; ++a)
            for (int b = 0; b < wr; ++b)
                for (int p = 0; p < dj; ++p)
                    for (int s = 0; s < dj; ++s) {
                        const double v = Wat(j, a, b, p, s);
                        ML[((size_t)p * wr + b) * (wl * dj) + a * dj + s] = v;   // (p v) <- (w s)
                        MR[((size_t)p * wl + a) * (wr * dj) + b * dj + s] = v;   // (p w) <- (v s)
                    }
        hl.push_back(dense_to_csr(ML, dj * wr, wl * dj));
        hr.push_back(dense_to_csr(MR, dj * wl, wr * dj));
    }
    for (int dd = 0; dd <= 8; ++dd) {
        std::vector<double> Id((size_t)dd * dd, 0.0);
        for (int i = 0; i < dd; ++i) Id[(size_t)i * dd + i] = 1.0;
        hi.push_back(dense_to_csr(Id, dd, dd));
    }
    // one device block for all CSR arrays
    std::vector<CsrHost> all;
    for (auto* v : {&hp, &hl, &hr, &hi}) all.insert(all.end(), v->begin(), v->end());
    std::vector<CsrDev> dv = upload_csr(c, all, &m->block);
    size_t k = 0;
    for (size_t i = 0; i < hp.size(); ++i) m->pair.push_back(dv[k++]);
    for (size_t i = 0; i < hl.size(); ++i) m->left.push_back(dv[k++]);
    for (size_t i = 0; i < hr.size(); ++i) m->right.push_back(dv[k++]);
    for (size_t i = 0; i < hi.size(); ++i) m->ident.push_back(dv[k++]);
    return m.release();
}

void mpo_destroy(ite_mpo* m) {
    if (!m) return;
    dev_free(m->ctx, m->block);
    delete m;
}

// ---------------------------------------------------------------------------
// MPS handle
// ---------------------------------------------------------------------------

std::vector<int> bond_caps(int L, const std::vector<int>& d, int chi_max) {
    std::vector<int> cap(L + 1);
    for (int b = 0; b <= L; ++b) {
        double left = 1.0, right = 1.0;
        for (int i = 0; i < b; ++i) left = std::min(left * d[i], 1e9);
        for (int i = b; i < L; ++i) right = std::min(right * d[i], 1e9);
        cap[b] = (int)std::min<double>(std::min(left, right), (double)chi_max);
    }
    return cap;
}

ite_mps* mps_new(ite_ctx* c, int L, const int* d, int chi_max) {
    ITE_REQUIRE(L >= 2, "mps: L must be >= 2");
    ITE_REQUIRE(chi_max >= 1, "mps: chi_max must be >= 1");
    ITE_REQUIRE(d != nullptr, "mps: NULL d");
    for (int i = 0; i < L; ++i) ITE_REQUIRE(d[i] >= 1 && d[i] <= 8, "mps: local dimension must be in 1..8");
    std::unique_ptr<ite_mps> p(new ite_mps);
    p->ctx = c;
    p->L = L;
    p->chi_max = chi_max;
    p->d.assign(d, d + L);
    p->Dcap = bond_caps(L, p->d, chi_max);
    p->D.assign(L + 1, 1);
    p->A.assign(L, nullptr);
    try {
        for (int i = 0; i < L; ++i)
            p->A[i] = static_cast<double*>(dev_alloc(c, (size_t)p->Dcap[i] * d[i] * p->Dcap[i + 1] * sizeof(double)));
    } catch (...) {
        for (double* a : p->A) dev_free(c, a);
        throw;
    }
    return p.release();
}

static void free_evolution(ite_mps* p) {
    ite_ctx* c = p->ctx;
    for (double* a : p->X) dev_free(c, a);
    p->X.clear();
    for (auto& e : p->env) {
        dev_free(c, e.H);
        dev_free(c, e.Hp);
        dev_free(c, e.O);
    }
    p->env.clear();
    p->env_w = 0;
}

void mps_destroy(ite_mps* p) {
    if (!p) return;
    ite_ctx* c = p->ctx;
    mps_destroy(p->aux);
    free_evolution(p);
    for (double* a : p->A) dev_free(c, a);
    delete p;
}

static void ensure_evolution(ite_mps* p, const ite_mpo* H) {
    ite_ctx* c = p->ctx;
    int wmax = 1;
    for (int v : H->w) wmax = std::max(wmax, v);
    if (!p->env.empty() && p->env_w >= wmax) return;
    free_evolution(p);
    const int L = p->L;
    p->X.assign(L, nullptr);
    for (int i = 0; i < L; ++i)
        p->X[i] = static_cast<double*>(dev_alloc(c, (size_t)p->Dcap[i] * p->d[i] * p->Dcap[i + 1] * sizeof(double)));
    p->env.assign(L + 1, BondEnv{});
    for (int b = 0; b <= L; ++b) {
        const size_t D = p->Dcap[b];
        p->env[b].H = static_cast<double*>(dev_alloc(c, D * wmax * D * sizeof(double)));
        p->env[b].Hp = static_cast<double*>(dev_alloc(c, D * wmax * D * sizeof(double)));
        p->env[b].O = static_cast<double*>(dev_alloc(c, D * D * sizeof(double)));
    }
    p->env_w = wmax;
}

// ---------------------------------------------------------------------------
// Energy and overlap
// ---------------------------------------------------------------------------

// <x|H|x> / <x|x> at the block (0, 1) with R = right environment at bond 2,
// x right-orthonormal from site 2 on.
static double centre_energy(ite_ctx* c, const ite_mpo* H, const std::vector<double*>& A, const std::vector<int>& D,
                            const double* R2) {
    const int d1 = H->d[0], d2 = H->d[1];
    const size_t n = (size_t)D[0] * d1 * d2 * D[2];
    double* th = slot_t<double>(c, SL_TMPA, n);
    double* y = slot_t<double>(c, SL_TMPB, n);
    two_site(c, D[0], d1, D[1], d2, D[2], A[0], A[1], th);
    double* L0 = slot_t<double>(c, SL_SMALL, 512) + 300;
    fill(L0, 1.0, 1, c->stream);
    HeffShape s{D[0], D[0], D[2], D[2], d1, d2, H->w[0], H->w[2]};
    heff_apply(c, s, L0, H->pair[0], R2, th, 1.0, 0.0, nullptr, y, Prec::F64);
    const double num = dot(c, th, y, n);
    const double den = dot(c, th, th, n);
    return num / den;
}

double measure_energy(ite_mps* psi, const ite_mpo* H) {
    ite_ctx* c = psi->ctx;
    ensure_evolution(psi, H);
    const int L = psi->L;
    auto& env = psi->env;
    fill(env[L].H, 1.0, 1, c->stream);
    for (int b = L - 1; b >= 2; --b)
        env_right(c, psi->D[b + 1], psi->D[b + 1], psi->D[b], psi->D[b], psi->d[b], H->w[b], H->w[b + 1],
                  env[b + 1].H, psi->A[b], &H->right[b], psi->A[b], env[b].H);
    return centre_energy(c, H, psi->A, psi->D, env[2].H);
}

double overlap(ite_mps* a, ite_mps* b) {
    ite_ctx* c = a->ctx;
    const int L = a->L;
    size_t mx = 1;
    for (int i = 0; i <= L; ++i) mx = std::max(mx, (size_t)a->D[i] * b->D[i]);
    double* E0 = slot_t<double>(c, SL_TMPA, mx);
    double* E1 = slot_t<double>(c, SL_TMPB, mx);
    fill(E0, 1.0, 1, c->stream);
    for (int i = 0; i < L; ++i) {
        env_left(c, a->D[i], b->D[i], a->D[i + 1], b->D[i + 1], a->d[i], 1, 1, E0, a->A[i], nullptr, b->A[i], E1);
        std::swap(E0, E1);
    }
    double* h = pinned(c, 64);
    d2h(c, h, E0, 1);
    sync(c);
    return h[0];
}

// ---------------------------------------------------------------------------
// The implicit step
// ---------------------------------------------------------------------------

namespace {
// Device-time spans of a step's phases, from the context's event pool (the
// caller resets the pool once per step or batch of steps).
struct Timer {
    ite_ctx* c;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> spans;
    explicit Timer(ite_ctx* cc) : c(cc) {}
    hipEvent_t ev() {
        if (c->events_used == c->events.size()) {
            hipEvent_t e;
            HIP_CHECK(hipEventCreate(&e));
            c->events.push_back(e);
        }
        return c->events[c->events_used++];
    }
    int open(int phase) {
        hipEvent_t a = ev(), b = ev();
        HIP_CHECK(hipEventRecord(a, c->stream));
        spans.push_back({phase, {a, b}});
        return (int)spans.size() - 1;
    }
    void close(int idx) { HIP_CHECK(hipEventRecord(spans[idx].second.second, c->stream)); }
    void collect(double* ms) {
        sync(c);
        for (auto& s : spans) {
            float t = 0.f;
            HIP_CHECK(hipEventElapsedTime(&t, s.second.first, s.second.second));
            ms[s.first] += t;
        }
    }
};
enum { PH_TOTAL = 0, PH_RHS, PH_SOLVE, PH_SPLIT, PH_ENV, PH_N };
}  // namespace

void check_step(const ite_mps* psi, const ite_mpo* H, double h, const ite_step_opts& o) {
    const int L = psi->L;
    ITE_REQUIRE(std::isfinite(h) && h > 0.0, "imag_step: h must be finite and > 0");
    if (H->L != L) ITE_FAIL(ITE_ESTATE, "imag_step: MPS and MPO lengths differ");
    for (int i = 0; i < L; ++i)
        if (H->d[i] != psi->d[i]) ITE_FAIL(ITE_ESTATE, "imag_step: local dimensions of MPS and MPO differ");
    ITE_REQUIRE(o.scheme == ITE_SCHEME_TRAP || o.scheme == ITE_SCHEME_BE || o.scheme == ITE_SCHEME_GL,
                "imag_step: unknown scheme");
    ITE_REQUIRE(o.scheme != ITE_SCHEME_GL || (o.gl_nodes >= 1 && o.gl_nodes <= 7),
                "imag_step: gl_nodes must be in 1..7");
    ITE_REQUIRE(o.rhs_mode == ITE_RHS_PROJECT || o.rhs_mode == ITE_RHS_MPS, "imag_step: unknown rhs_mode");
    ITE_REQUIRE(o.shift_mode == ITE_SHIFT_FIXED || o.shift_mode == ITE_SHIFT_TRACK, "imag_step: unknown shift mode");
    ITE_REQUIRE(std::isfinite(o.shift), "imag_step: non-finite shift");
    ITE_REQUIRE(o.chi_max >= 1, "imag_step: chi_max must be >= 1");
    ITE_REQUIRE(o.cutoff >= 0.0 && o.cutoff < 1.0, "imag_step: cutoff must be in [0, 1)");
    ITE_REQUIRE(o.tie_rel >= 0.0, "imag_step: tie_rel must be >= 0");
    ITE_REQUIRE(o.krylov_dim >= 1 && o.krylov_dim <= 64, "imag_step: krylov_dim must be in 1..64");
    ITE_REQUIRE(o.max_cycles >= 1, "imag_step: max_cycles must be >= 1");
    ITE_REQUIRE(o.tol_loc >= 0.0, "imag_step: tol_loc must be >= 0");
    ITE_REQUIRE(o.nsweeps >= 1, "imag_step: nsweeps must be >= 1");
    ITE_REQUIRE(o.precision >= 0 && o.precision <= 2, "imag_step: unknown precision");
    ITE_REQUIRE(o.precision == ITE_PREC_FP64 || (o.max_refine >= 0 && o.tol_refine >= 0.0),
                "imag_step: mixed precision needs max_refine >= 0 and tol_refine >= 0");
    ITE_REQUIRE(o.init_guess == ITE_GUESS_PSI || o.init_guess == ITE_GUESS_B, "imag_step: unknown init_guess");
}

// One implicit step of one state, split into the phases of a block so that a
// batch of states can sweep in lockstep (step_batch): the constructor does
// the step's set-up (shift, x <- psi, right environments), then for every
// slot of the sweep rhs() forms b and the initial guess of the block,
// solve() (or a batched solve) the local problem, split_env() the split and
// the environment updates; finish() normalises and replaces psi.
struct StepRun {
    ite_mps* psi;
    const ite_mpo* H;
    ite_step_opts o;
    ite_ctx* c;
    int L, chi, refine, nblocks;
    double h, s, acoef;
    Timer tm;
    int t_all = -1;
    ite_step_report r{};
    int nres = 0;
    double sum_res = 0.0;
    double* stats_dev;
    std::vector<char> deferred;
    bool guess_b;
    // the block of the current slot
    int bi = 0, bdir = 0, blk = 0;
    double* bvec = nullptr;
    double* th = nullptr;
    LocalOp op;

    StepRun(ite_mps* p, const ite_mpo* Hm, double hh, const ite_step_opts& oo, double* stats)
        : psi(p), H(Hm), o(oo), c(p->ctx), h(hh), tm(p->ctx), stats_dev(stats) {
        check_step(psi, H, h, o);
        ensure_evolution(psi, H);
        L = psi->L;
        nblocks = 2 * (L - 1) * o.nsweeps;
        t_all = tm.open(PH_TOTAL);
        s = o.shift;
        if (o.shift_mode == ITE_SHIFT_TRACK) {
            if (!psi->e_valid) {
                psi->energy = measure_energy(psi, H);
                psi->e_valid = true;
            }
            s = psi->energy;
        }
        chi = std::min(o.chi_max, psi->chi_max);
        auto& env = psi->env;
        auto& X = psi->X;
        auto& XD = psi->XD;
        const auto& P = psi->A;
        const auto& PD = psi->D;
        XD = PD;
        for (int i = 0; i < L; ++i) d2d(c, X[i], P[i], (size_t)PD[i] * psi->d[i] * PD[i + 1]);
        // boundary environments
        fill(env[0].H, 1.0, 1, c->stream);
        fill(env[0].Hp, 1.0, 1, c->stream);
        fill(env[0].O, 1.0, 1, c->stream);
        fill(env[L].H, 1.0, 1, c->stream);
        fill(env[L].Hp, 1.0, 1, c->stream);
        fill(env[L].O, 1.0, 1, c->stream);
        env[0].hp_alias = env[0].o_ident = false;
        env[L].hp_alias = env[L].o_ident = false;
        for (int b = L - 1; b >= 2; --b) {
            env_right(c, XD[b + 1], XD[b + 1], XD[b], XD[b], psi->d[b], H->w[b], H->w[b + 1], env[b + 1].H, X[b],
                      &H->right[b], X[b], env[b].H);
        }
        for (int b = 2; b < L; ++b) {
            env[b].hp_alias = true;
            env[b].o_ident = true;
        }
        r.h = h;
        r.shift = s;
        r.dtau = o.scheme == ITE_SCHEME_TRAP ? 2.0 * h : h;
        acoef = 1.0 - h * s;
        // refinement rounds: 0 picks the cheapest count that keeps the step
        // within 1e-8 relative energy of the FP64 step at the fixed budget
        // (measured: FP32 operands 1e-12 after one correction; BF16 operands
        // 3e-7 after one, 1e-10 after two)
        refine = o.max_refine > 0 ? o.max_refine : (o.precision == ITE_PREC_BF16_IR ? 2 : 1);
        // Appendix B: the right-hand side is the initial guess of the solve; in
        // x's (= psi's) basis that is b_loc itself on the step's first block
        guess_b = o.init_guess == ITE_GUESS_B;
        deferred.assign(nblocks, 0);
    }

    // Sweep order: left to right, then right to left, nsweeps times.
    void slot_block(int slot, int& i, int& dir) const {
        const int t = slot % (2 * (L - 1));
        if (t < L - 1) {
            i = t;
            dir = 0;
        } else {
            i = L - 2 - (t - (L - 1));
            dir = 1;
        }
    }
    size_t block_n(int slot) const {
        int i, dir;
        slot_block(slot, i, dir);
        return (size_t)psi->XD[i] * psi->d[i] * psi->d[i + 1] * psi->XD[i + 2];
    }
    // A local solve the batched GMRES takes: fixed budget, Krylov dimension
    // below the vector length and at most 16; FP64, or FP32 refinement with a
    // fixed number of corrections of one GMRES cycle each (the batch then
    // runs one cycle per correction).
    bool batchable(int slot) const {
        int i, dir;
        slot_block(slot, i, dir);
        const int I = H->w[i] * psi->d[i] * psi->d[i + 1];
        const bool prec_ok = o.precision == ITE_PREC_FP64 ||
                             (o.precision == ITE_PREC_FP32_IR && o.tol_refine <= 0.0 && o.max_cycles == 1);
        return prec_ok && o.tol_loc <= 0.0 && o.krylov_dim <= 16 && (size_t)o.krylov_dim < block_n(slot) &&
               I <= BATCH_STAGE_SC;
    }
    // The batch's cycles and precision for a batchable solve.
    bool batch_lo() const { return o.precision != ITE_PREC_FP64; }
    int batch_cycles() const { return batch_lo() ? refine : o.max_cycles; }

    // b and the initial guess of the slot's block into bv and thv (length
    // block_n); sets op.
    void rhs(int slot, double* bv, double* thv) {
        slot_block(slot, bi, bdir);
        blk = slot;
        bvec = bv;
        th = thv;
        const int i = bi;
        auto& env = psi->env;
        auto& X = psi->X;
        auto& XD = psi->XD;
        const auto& P = psi->A;
        const auto& PD = psi->D;
        const int d1 = psi->d[i], d2 = psi->d[i + 1];
        const int Dl = XD[i], Dr = XD[i + 2], Dpl = PD[i], Dpr = PD[i + 2];
        const size_t npsi = (size_t)Dpl * d1 * d2 * Dpr;
        const size_t nx = (size_t)Dl * d1 * d2 * Dr;
        double* tpsi = slot_t<double>(c, SL_TPSI, npsi);
        const int t_rhs = tm.open(PH_RHS);
        two_site(c, Dpl, d1, PD[i + 1], d2, Dpr, P[i], P[i + 1], tpsi);
        const double* Lo = env[i].o_ident ? nullptr : env[i].O;
        const double* Ro = env[i + 2].o_ident ? nullptr : env[i + 2].O;
        const double ovc = o.scheme == ITE_SCHEME_TRAP ? 1.0 + h * s : 1.0;
        overlap_apply(c, Dl, Dpl, Dr, Dpr, d1, d2, Lo, Ro, tpsi, ovc, bvec);
        if (o.scheme == ITE_SCHEME_TRAP) {
            const double* Lh = env[i].hp_alias ? env[i].H : env[i].Hp;
            const double* Rh = env[i + 2].hp_alias ? env[i + 2].H : env[i + 2].Hp;
            HeffShape hs{Dl, Dpl, Dr, Dpr, d1, d2, H->w[i], H->w[i + 2]};
            heff_apply(c, hs, Lh, H->pair[i], Rh, tpsi, -h, 1.0, bvec, bvec, Prec::F64);
        }
        if (guess_b) d2d(c, th, bvec, nx);
        else two_site(c, Dl, d1, XD[i + 1], d2, Dr, X[i], X[i + 1], th);
        guess_b = false;
        tm.close(t_rhs);
        op.s = HeffShape{Dl, Dl, Dr, Dr, d1, d2, H->w[i], H->w[i + 2]};
        op.L = env[i].H;
        op.R = env[i + 2].H;
        op.ww = &H->pair[i];
        op.alpha = acoef;
        op.beta = h;
    }
    double* stats_of(int slot) const { return stats_dev + (size_t)8 * slot; }

    void solve() {
        const int t_solve = tm.open(PH_SOLVE);
        SolveStats ss = local_solve(c, op, bvec, th, o.krylov_dim, o.max_cycles, o.tol_loc, o.precision, refine,
                                    o.tol_refine, stats_of(blk));
        tm.close(t_solve);
        if (ss.deferred) deferred[blk] = 1;
        else add(ss);
    }
    void add(const SolveStats& ss) {
        r.matvecs_fp64 += ss.matvecs64;
        r.matvecs_lo += ss.matvecs_lo;
        r.flags |= ss.flags;
        r.max_res_rel = std::max(r.max_res_rel, ss.res_rel);
        sum_res += ss.res_rel;
        ++nres;
    }

    void split_env() {
        const int i = bi;
        auto& env = psi->env;
        auto& X = psi->X;
        auto& XD = psi->XD;
        const auto& P = psi->A;
        const auto& PD = psi->D;
        const int d1 = psi->d[i], d2 = psi->d[i + 1];
        const int t_split = tm.open(PH_SPLIT);
        SplitResult sp = split(c, bdir, XD[i], d1, d2, XD[i + 2], th, chi, o.cutoff, o.tie_rel, X[i], X[i + 1],
                               nullptr);
        tm.close(t_split);
        XD[i + 1] = sp.k;
        r.max_disc = std::max(r.max_disc, sp.disc);
        r.sum_disc += sp.disc;
        if (bdir == 0 && i + 2 < L) {
            const int t_env = tm.open(PH_ENV);
            const int b = i + 1;
            // <x|H|x>, <x|H|psi>, <x|psi> at bond i+1 from bond i
            env_left(c, XD[i], XD[i], XD[b], XD[b], psi->d[i], H->w[i], H->w[b], env[i].H, X[i], &H->left[i], X[i],
                     env[b].H);
            const double* Ehp = env[i].hp_alias ? env[i].H : env[i].Hp;
            env_left(c, XD[i], PD[i], XD[b], PD[b], psi->d[i], H->w[i], H->w[b], Ehp, X[i], &H->left[i], P[i],
                     env[b].Hp);
            env_left(c, XD[i], PD[i], XD[b], PD[b], psi->d[i], 1, 1, env[i].O, X[i], nullptr, P[i], env[b].O);
            env[b].hp_alias = false;
            env[b].o_ident = false;
            tm.close(t_env);
        } else if (bdir == 1 && i > 0) {
            const int t_env = tm.open(PH_ENV);
            const int b = i + 1, a = i + 2;
            env_right(c, XD[a], XD[a], XD[b], XD[b], psi->d[b], H->w[b], H->w[a], env[a].H, X[b], &H->right[b], X[b],
                      env[b].H);
            const double* Ehp = env[a].hp_alias ? env[a].H : env[a].Hp;
            env_right(c, XD[a], PD[a], XD[b], PD[b], psi->d[b], H->w[b], H->w[a], Ehp, X[b], &H->right[b], P[b],
                      env[b].Hp);
            if (env[a].o_ident) {
                // <x|psi> with identity to the right: plain overlap of the site tensors
                double* Eid = slot_t<double>(c, SL_TMPA, (size_t)XD[a] * XD[a]);
                eye(Eid, XD[a], c->stream);
                env_right_overlap_pub(c, H->ident[psi->d[b]], XD[a], PD[a], XD[b], PD[b], psi->d[b], Eid, X[b], P[b],
                                      env[b].O);
            } else {
                env_right_overlap_pub(c, H->ident[psi->d[b]], XD[a], PD[a], XD[b], PD[b], psi->d[b], env[a].O, X[b],
                                      P[b], env[b].O);
            }
            env[b].hp_alias = false;
            env[b].o_ident = false;
            tm.close(t_env);
        }
    }

    // The records of the deferred solves (read by the caller into `host`).
    bool any_deferred() const { return std::find(deferred.begin(), deferred.end(), 1) != deferred.end(); }
    void add_deferred(const double* host) {
        for (int k = 0; k < nblocks; ++k)
            if (deferred[k]) add(stats_from(host + (size_t)8 * k, false, batch_lo()));
    }

    // Normalise the centre, measure, psi <- x.  Throws ENONFINITE (psi
    // unchanged) for a non-finite state.
    void finish(ite_step_report* rep) {
        auto& X = psi->X;
        auto& XD = psi->XD;
        // normalise the centre (site 1) and measure
        const size_t n0 = (size_t)XD[0] * psi->d[0] * XD[1];
        const double nrm2 = dot(c, X[0], X[0], n0);
        const double nrm = std::sqrt(std::max(nrm2, 0.0));
        bool finite = std::isfinite(nrm) && nrm > 0.0;
        double E = 0.0;
        if (finite) {
            scale(X[0], 1.0 / nrm, n0, c->stream);
            E = centre_energy(c, H, X, XD, psi->env[2].H);
            finite = std::isfinite(E);
        }
        tm.close(t_all);
        double ms[PH_N] = {0, 0, 0, 0, 0};
        tm.collect(ms);
        if (!finite) ITE_FAIL(ITE_ENONFINITE, "imag_step: non-finite state; psi left unchanged");
        // psi <- x
        std::swap(psi->A, psi->X);
        std::swap(psi->D, psi->XD);
        psi->tau += r.dtau;
        psi->energy = E;
        psi->e_valid = true;
        r.tau = psi->tau;
        r.energy = E;
        r.norm_before = nrm;
        r.max_chi = *std::max_element(psi->D.begin(), psi->D.end());
        r.mean_res_rel = nres ? sum_res / nres : 0.0;
        r.ms_total = ms[PH_TOTAL];
        r.ms_rhs = ms[PH_RHS];
        r.ms_solve = ms[PH_SOLVE];
        r.ms_split = ms[PH_SPLIT];
        r.ms_env = ms[PH_ENV];
        if (rep) *rep = r;
    }
};

void imag_step_sweep(ite_mps* psi, const ite_mpo* H, double h, const ite_step_opts& o, ite_step_report* rep) {
    ite_ctx* c = psi->ctx;
    check_step(psi, H, h, o);
    c->events_used = 0;
    const int nblocks = 2 * (psi->L - 1) * o.nsweeps;
    StepRun run(psi, H, h, o, slot_t<double>(c, SL_STATS, (size_t)8 * nblocks + 8));
    for (int slot = 0; slot < run.nblocks; ++slot) {
        const size_t nx = run.block_n(slot);
        run.rhs(slot, slot_t<double>(c, SL_B, nx), slot_t<double>(c, SL_TH, nx));
        run.solve();
        run.split_env();
    }
    if (run.any_deferred()) {
        double* host = pinned(c, (size_t)8 * nblocks + 64);
        d2h(c, host, run.stats_dev, (size_t)8 * nblocks);
        sync(c);
        run.add_deferred(host);
    }
    run.finish(rep);
}

// A batch of steps in lockstep: every state's sweep advances one block slot
// at a time; the slot's right-hand sides and guesses are formed state by
// state, the local solves that the batched GMRES takes run together
// (gmres_batch), the others one by one, then every state splits and updates
// its environments.  States with shorter sweeps drop out when theirs end.
// The per-state buffers of b and the guess persist across the phases of a
// slot, so they are carved per state from one slot of the context.
void step_batch(int n, ite_mps* const* psi, const ite_mpo* const* H, const double* h,
                const ite_step_opts* const* opts, ite_step_report* reps, int* status) {
    ITE_REQUIRE(n >= 1, "step_batch: n must be >= 1");
    ite_ctx* c = psi[0]->ctx;
    for (int j = 0; j < n; ++j) {
        ITE_REQUIRE(psi[j] && H[j] && opts[j], "step_batch: NULL state, Hamiltonian or options");
        if (psi[j]->ctx != c || H[j]->ctx != c) ITE_FAIL(ITE_ESTATE, "step_batch: every object must share one context");
        for (int q = 0; q < j; ++q)
            if (psi[q] == psi[j]) ITE_FAIL(ITE_EINVAL, "step_batch: a state appears twice");
        check_step(psi[j], H[j], h[j], *opts[j]);
    }
    // panels and MPS right-hand sides are whole-state operations: one by one,
    // the plain sweeps of the others in lockstep
    std::vector<int> plain;
    for (int j = 0; j < n; ++j) {
        if (!step_is_composite(*opts[j])) {
            plain.push_back(j);
            continue;
        }
        try {
            imag_step(psi[j], H[j], h[j], *opts[j], reps ? &reps[j] : nullptr);
            if (status) status[j] = ITE_OK;
        } catch (const Error& e) {
            if (!status) throw;
            status[j] = e.code;
            c->err = e.what();
        }
    }
    if ((int)plain.size() < n) {
        if (plain.empty()) return;
        const int m = (int)plain.size();
        std::vector<ite_mps*> ps(m);
        std::vector<const ite_mpo*> hs(m);
        std::vector<double> hh(m);
        std::vector<const ite_step_opts*> os(m);
        std::vector<ite_step_report> rs(m);
        std::vector<int> st(m, ITE_OK);
        for (int q = 0; q < m; ++q) {
            ps[q] = psi[plain[q]];
            hs[q] = H[plain[q]];
            hh[q] = h[plain[q]];
            os[q] = opts[plain[q]];
        }
        step_batch(m, ps.data(), hs.data(), hh.data(), os.data(), rs.data(), status ? st.data() : nullptr);
        for (int q = 0; q < m; ++q) {
            if (reps) reps[plain[q]] = rs[q];
            if (status) status[plain[q]] = st[q];
        }
        return;
    }
    c->events_used = 0;
    // per-state records and b / guess buffers
    std::vector<size_t> soff(n), boff(n), bmax(n);
    size_t stot = 0, btot = 0;
    for (int j = 0; j < n; ++j) {
        const ite_mps* p = psi[j];
        size_t mx = 1;
        for (int i = 0; i + 1 < p->L; ++i)
            mx = std::max(mx, (size_t)p->Dcap[i] * p->d[i] * p->d[i + 1] * p->Dcap[i + 2]);
        bmax[j] = (mx + 31) & ~size_t(31);
        boff[j] = btot;
        btot += 2 * bmax[j];
        soff[j] = stot;
        stot += (size_t)8 * 2 * (p->L - 1) * opts[j]->nsweeps + 32;
    }
    double* sbase = slot_t<double>(c, SL_STATS, stot);
    double* bbase = slot_t<double>(c, SL_BATCHB, btot);
    std::vector<std::unique_ptr<StepRun>> runs(n);
    int maxslots = 0;
    for (int j = 0; j < n; ++j) {
        runs[j].reset(new StepRun(psi[j], H[j], h[j], *opts[j], sbase + soff[j]));
        maxslots = std::max(maxslots, runs[j]->nblocks);
    }
    // batches by budget (Krylov dimension, cycles) and precision
    for (int slot = 0; slot < maxslots; ++slot) {
        std::map<std::tuple<int, int, bool>, std::vector<int>> groups;
        for (int j = 0; j < n; ++j) {
            StepRun& r = *runs[j];
            if (slot >= r.nblocks) continue;
            double* bv = bbase + boff[j];
            r.rhs(slot, bv, bv + bmax[j]);
            if (r.batchable(slot)) groups[std::make_tuple(r.o.krylov_dim, r.batch_cycles(), r.batch_lo())].push_back(j);
            else r.solve();
        }
        for (auto& grp : groups) {
            std::vector<BatchItem> items;
            std::vector<int> spans;
            for (int j : grp.second) {
                StepRun& r = *runs[j];
                items.push_back(BatchItem{r.op, r.bvec, r.th, r.stats_of(slot)});
                r.deferred[slot] = 1;
                spans.push_back(r.tm.open(PH_SOLVE));
            }
            gmres_batch(c, items, std::get<0>(grp.first), std::get<1>(grp.first), std::get<2>(grp.first));
            for (size_t q = 0; q < grp.second.size(); ++q) runs[grp.second[q]]->tm.close(spans[q]);
        }
        for (int j = 0; j < n; ++j)
            if (slot < runs[j]->nblocks) runs[j]->split_env();
    }
    bool any = false;
    for (int j = 0; j < n; ++j) any = any || runs[j]->any_deferred();
    if (any) {
        double* host = pinned(c, stot + 64);
        d2h(c, host, sbase, stot);
        sync(c);
        for (int j = 0; j < n; ++j) runs[j]->add_deferred(host + soff[j]);
    }
    for (int j = 0; j < n; ++j) {
        try {
            runs[j]->finish(reps ? &reps[j] : nullptr);
            if (status) status[j] = ITE_OK;
        } catch (const Error& e) {
            if (!status) throw;
            status[j] = e.code;
            c->err = e.what();
        }
    }
}

// ---------------------------------------------------------------------------
// DMRG ground-state sweeps
// ---------------------------------------------------------------------------

// Lowest eigenpair of the symmetric operator op by the Lanczos method with
// full reorthogonalisation: the Arnoldi steps of the GMRES solver (classical
// Gram-Schmidt twice), the projected matrix diagonalised on the device
// (lanczos_eig), x = V y, and a restart from that Ritz vector, for at most
// max_cycles cycles of m steps or until ||op x - theta x|| <= tol |theta|
// (estimated as |h_(k+1,k) y_k|).  x: the start vector on entry (any norm),
// the normalised Ritz vector on return.  rec (device, 4 doubles, zeroed
// here): [0] theta, [1] relative residual, [2] products, [3] steps of the
// last cycle.  With one cycle nothing waits for the host; more cycles read
// rec once per cycle for the stopping test.
static void lanczos_lowest(ite_ctx* c, const LocalOp& op, double* x, int m, int max_cycles, double tol,
                           double* rec) {
    const size_t n = op.n();
    const int mm = (int)std::min<size_t>((size_t)m, n);
    constexpr int HC = HESS_HC;   // per column: [0,64) first-pass coefficients, [64,128) second pass, 128 norm
    double* V = slot_t<double>(c, SL_V, (size_t)(mm + 1) * n);
    double* w = slot_t<double>(c, SL_W, n);
    const int nb = reduce_blocks(n);
    double* part = slot_t<double>(c, SL_PART, (size_t)nb * 64 + 64);
    double* hd = slot_t<double>(c, SL_HESS, (size_t)mm * HC + 8 + 64);
    double* xnorm_d = hd + (size_t)mm * HC;
    double* ydev = hd + (size_t)mm * HC + 8;
    fill(rec, 0.0, 4, c->stream);
    for (int cyc = 0; cyc < max_cycles; ++cyc) {
        dot_partials(x, x, n, part, c->stream);
        finish_partials(part, 1, nb, xnorm_d, 2, c->stream);
        scale_inv(x, xnorm_d, V, n, c->stream);
        for (int k = 0; k < mm; ++k) {
            double* col = hd + (size_t)k * HC;
            double* vnext = k + 1 < mm ? V + (size_t)(k + 1) * n : nullptr;
            op_apply(c, op, V + (size_t)k * n, w);
            if (cgs2_small(V, (long)n, k + 1, w, n, col, vnext, c->stream)) continue;
            mdot_partials(V, (long)n, k + 1, w, n, part, c->stream);
            finish_partials(part, k + 1, nb, col, 0, c->stream);
            gemv_sub(V, (long)n, k + 1, col, w, n, c->stream);
            mdot_partials(V, (long)n, k + 1, w, n, part, c->stream);
            finish_partials(part, k + 1, nb, col + 64, 0, c->stream);
            gemv_sub(V, (long)n, k + 1, col + 64, w, n, c->stream);
            dot_partials(w, w, n, part, c->stream);
            finish_partials(part, 1, nb, col + 128, 2, c->stream);
            if (vnext) scale_inv(w, col + 128, vnext, n, c->stream);
        }
        lanczos_eig(hd, mm, ydev, rec, c->stream);
        fill(x, 0.0, n, c->stream);
        gemv_add(V, (long)n, mm, ydev, x, n, c->stream);
        if (cyc + 1 < max_cycles) {
            double* host = pinned(c, 64);
            d2h(c, host, rec, 4);
            sync(c);
            if (!std::isfinite(host[0])) ITE_FAIL(ITE_ENONFINITE, "dmrg: non-finite Ritz value");
            const bool converged = host[0] != 0.0 ? host[1] <= tol : host[1] == 0.0;
            if ((int)host[3] < mm || converged) break;
        }
    }
}

void dmrg_sweeps(ite_mps* psi, const ite_mpo* H, const DmrgOpts& o, DmrgReport* rep) {
    ite_ctx* c = psi->ctx;
    const int L = psi->L;
    if (H->L != L) ITE_FAIL(ITE_ESTATE, "dmrg: MPS and MPO lengths differ");
    for (int i = 0; i < L; ++i)
        if (H->d[i] != psi->d[i]) ITE_FAIL(ITE_ESTATE, "dmrg: local dimensions of MPS and MPO differ");
    ITE_REQUIRE(o.nsweeps >= 1, "dmrg: nsweeps must be >= 1");
    ITE_REQUIRE(o.chi_max >= 1, "dmrg: chi_max must be >= 1");
    ITE_REQUIRE(o.cutoff >= 0.0 && o.cutoff < 1.0, "dmrg: cutoff must be in [0, 1)");
    ITE_REQUIRE(o.tie_rel >= 0.0, "dmrg: tie_rel must be >= 0");
    ITE_REQUIRE(o.krylov_dim >= 1 && o.krylov_dim <= 64, "dmrg: krylov_dim must be in 1..64");
    ITE_REQUIRE(o.max_cycles >= 1, "dmrg: max_cycles must be >= 1");
    ITE_REQUIRE(o.tol >= 0.0, "dmrg: tol must be >= 0");
    ensure_evolution(psi, H);
    const int chi = std::min(o.chi_max, psi->chi_max);
    auto& env = psi->env;
    auto& X = psi->X;
    auto& XD = psi->XD;
    XD = psi->D;
    for (int i = 0; i < L; ++i) d2d(c, X[i], psi->A[i], (size_t)psi->D[i] * psi->d[i] * psi->D[i + 1]);
    fill(env[0].H, 1.0, 1, c->stream);
    fill(env[L].H, 1.0, 1, c->stream);
    for (int b = L - 1; b >= 2; --b)
        env_right(c, XD[b + 1], XD[b + 1], XD[b], XD[b], psi->d[b], H->w[b], H->w[b + 1], env[b + 1].H, X[b],
                  &H->right[b], X[b], env[b].H);
    DmrgReport r{};
    const int nblocks = 2 * (L - 1) * o.nsweeps;
    double* recs = slot_t<double>(c, SL_STATS, (size_t)4 * nblocks + 8);
    int blk = 0;
    auto block = [&](int i, int dir) {
        const int d1 = psi->d[i], d2 = psi->d[i + 1];
        const int Dl = XD[i], Dr = XD[i + 2];
        double* th = slot_t<double>(c, SL_TH, (size_t)Dl * d1 * d2 * Dr);
        two_site(c, Dl, d1, XD[i + 1], d2, Dr, X[i], X[i + 1], th);
        LocalOp op;
        op.s = HeffShape{Dl, Dl, Dr, Dr, d1, d2, H->w[i], H->w[i + 2]};
        op.L = env[i].H;
        op.R = env[i + 2].H;
        op.ww = &H->pair[i];
        op.alpha = 0.0;
        op.beta = 1.0;
        lanczos_lowest(c, op, th, o.krylov_dim, o.max_cycles, o.tol, recs + (size_t)4 * blk);
        ++blk;
        const SplitResult sp = split(c, dir, Dl, d1, d2, Dr, th, chi, o.cutoff, o.tie_rel, X[i], X[i + 1], nullptr);
        XD[i + 1] = sp.k;
        r.max_disc = std::max(r.max_disc, sp.disc);
    };
    for (int sw = 0; sw < o.nsweeps; ++sw) {
        for (int i = 0; i + 1 < L; ++i) {
            block(i, 0);
            if (i + 2 < L)
                env_left(c, XD[i], XD[i], XD[i + 1], XD[i + 1], psi->d[i], H->w[i], H->w[i + 1], env[i].H, X[i],
                         &H->left[i], X[i], env[i + 1].H);
        }
        for (int i = L - 2; i >= 0; --i) {
            block(i, 1);
            if (i > 0)
                env_right(c, XD[i + 2], XD[i + 2], XD[i + 1], XD[i + 1], psi->d[i + 1], H->w[i + 1], H->w[i + 2],
                          env[i + 2].H, X[i + 1], &H->right[i + 1], X[i + 1], env[i + 1].H);
        }
    }
    {
        double* host = pinned(c, (size_t)4 * nblocks + 64);
        d2h(c, host, recs, (size_t)4 * nblocks);
        sync(c);
        for (int k = 0; k < nblocks; ++k) {
            const double* rc = host + (size_t)4 * k;
            if (!std::isfinite(rc[0])) ITE_FAIL(ITE_ENONFINITE, "dmrg: non-finite Ritz value");
            r.matvecs += (long long)rc[2];
            r.max_res_rel = std::max(r.max_res_rel, rc[1]);
        }
    }
    // the mixed environments of the evolution describe the previous state
    for (int b = 2; b < L; ++b) {
        env[b].hp_alias = true;
        env[b].o_ident = true;
    }
    // normalise the centre (site 1; the last eigenvector is normalised, the
    // truncation of its split may not be) and measure
    const size_t n0 = (size_t)XD[0] * psi->d[0] * XD[1];
    const double nrm = std::sqrt(std::max(dot(c, X[0], X[0], n0), 0.0));
    if (!(std::isfinite(nrm) && nrm > 0.0)) ITE_FAIL(ITE_ENONFINITE, "dmrg: non-finite state; psi left unchanged");
    scale(X[0], 1.0 / nrm, n0, c->stream);
    const double E = centre_energy(c, H, X, XD, env[2].H);
    if (!std::isfinite(E)) ITE_FAIL(ITE_ENONFINITE, "dmrg: non-finite energy; psi left unchanged");
    std::swap(psi->A, psi->X);
    std::swap(psi->D, psi->XD);
    psi->energy = E;
    psi->e_valid = true;
    r.energy = E;
    r.max_chi = *std::max_element(psi->D.begin(), psi->D.end());
    if (rep) *rep = r;
}

// ---------------------------------------------------------------------------
// One-site expectation values (the observable of the METTS chains)
// ---------------------------------------------------------------------------

// <psi|O_site|psi> / <psi|psi>: the overlap transfer from the left up to the
// site (E[a', a] over sites < site), T = E A_site (GEMM), U = O T on the
// physical index (a GEMM batched over the left index), then the two
// contractions A . U and A . T.  The sites right of `site` are
// right-orthonormal in every state this library leaves (centre on site 1),
// so they contribute the identity.
double site_expect(ite_mps* psi, int site, const double* op_host) {
    ite_ctx* c = psi->ctx;
    const int L = psi->L;
    ITE_REQUIRE(site >= 0 && site < L, "expect_site: site out of range");
    const int d = psi->d[site];
    for (int k = 0; k < d * d; ++k) ITE_REQUIRE(std::isfinite(op_host[k]), "expect_site: non-finite operator entry");
    size_t mx = 1;
    for (int i = 0; i <= site; ++i) mx = std::max(mx, (size_t)psi->D[i] * psi->D[i]);
    double* E0 = slot_t<double>(c, SL_TMPA, mx);
    double* E1 = slot_t<double>(c, SL_TMPB, mx);
    fill(E0, 1.0, 1, c->stream);
    for (int i = 0; i < site; ++i) {
        env_left(c, psi->D[i], psi->D[i], psi->D[i + 1], psi->D[i + 1], psi->d[i], 1, 1, E0, psi->A[i], nullptr,
                 psi->A[i], E1);
        std::swap(E0, E1);
    }
    const int Dl = psi->D[site], Dr = psi->D[site + 1];
    const size_t n = (size_t)Dl * d * Dr;
    double* T = slot_t<double>(c, SL_R64, n);
    double* U = slot_t<double>(c, SL_D64, n);
    double* op = slot_t<double>(c, SL_SMALL, 512) + 320;   // d <= 8: 64 values
    h2d(c, op, op_host, sizeof(double) * d * d);
    gemm(c, false, false, Dl, d * Dr, Dl, 1.0, E0, Dl, psi->A[site], (long)d * Dr, 0.0, nullptr, 0, T, (long)d * Dr);
    Gemm g;
    g.M = d; g.N = Dr; g.K = d;
    g.A = op; g.lda = d; g.sA = 0;
    g.B = T; g.ldb = Dr; g.sB = (long)d * Dr;
    g.D = U; g.ldd = Dr; g.sD = (long)d * Dr;
    g.batch = Dl;
    gemm_f64(g, c->stream);
    const double num = dot(c, psi->A[site], U, n);
    const double den = dot(c, psi->A[site], T, n);
    ITE_REQUIRE(den > 0.0 && std::isfinite(den), "expect_site: zero or non-finite state");
    return num / den;
}

// ---------------------------------------------------------------------------
// Product-basis sampling (METTS collapse)
// ---------------------------------------------------------------------------

// Site by site from the left, all samples at once: T = V A_i (FP64 GEMM,
// V [S][D_i] the samples' normalised left vectors), then one workgroup per
// sample picks s_i from the conditional probabilities ||T[smp][s]||^2 (exact
// because the sites right of i are right-orthonormal) and forms the next V.
// Device buffers: u [L][S] uniforms, cfg [S][L] output, V0 and V1
// [S][D_max], T [S][d_max][D_max], flag [2] (zeroed here; [0] set for a zero
// or non-finite total, [1] for a uniform outside [0, 1)).
void mps_sample_core(ite_mps* psi, int S, const double* u, int* cfg, double* V0, double* V1, double* T,
                     double* flag) {
    ite_ctx* c = psi->ctx;
    const int L = psi->L;
    fill(V0, 1.0, (size_t)S, c->stream);
    fill(flag, 0.0, 2, c->stream);
    for (int i = 0; i < L; ++i) {
        const int Dl = psi->D[i], Dr = psi->D[i + 1], d = psi->d[i];
        gemm(c, false, false, S, d * Dr, Dl, 1.0, V0, Dl, psi->A[i], (long)d * Dr, 0.0, nullptr, 0, T,
             (long)d * Dr);
        sample_site(T, S, d, Dr, u + (size_t)i * S, V1, cfg, L, i, flag, c->stream);
        std::swap(V0, V1);
    }
}

size_t mps_sample_scratch_doubles(const ite_mps* psi, int S) {
    int Dmax = 1, dmax = 1;
    for (int i = 0; i < psi->L; ++i) {
        Dmax = std::max(Dmax, psi->D[i + 1]);
        dmax = std::max(dmax, psi->d[i]);
    }
    return 32 + (size_t)S * Dmax * (2 + dmax);
}

static void sample_flags(double f0, double f1) {
    if (f1 != 0.0) ITE_FAIL(ITE_EINVAL, "mps_sample: uniforms must lie in [0, 1)");
    if (f0 != 0.0)
        ITE_FAIL(ITE_ENONFINITE, "mps_sample: a conditional probability had a zero or non-finite total "
                                 "(the state is zero or not finite)");
}

void mps_sample(ite_mps* psi, int S, const double* uniforms, int* configs) {
    ite_ctx* c = psi->ctx;
    const int L = psi->L;
    ITE_REQUIRE(S >= 1, "mps_sample: nsamples must be >= 1");
    for (size_t k = 0; k < (size_t)S * L; ++k)
        ITE_REQUIRE(uniforms[k] >= 0.0 && uniforms[k] < 1.0, "mps_sample: uniforms must lie in [0, 1)");
    const size_t nw = mps_sample_scratch_doubles(psi, S);
    double* ws = slot_t<double>(c, SL_X1, nw);
    double* u = slot_t<double>(c, SL_PART, (size_t)S * L);
    int* cfg = slot_t<int>(c, SL_PERM, (size_t)S * L);
    double* flag = ws;
    int Dmax = 1;
    for (int i = 0; i < L; ++i) Dmax = std::max(Dmax, psi->D[i + 1]);
    double* V0 = ws + 32;
    double* V1 = V0 + (size_t)S * Dmax;
    double* T = V1 + (size_t)S * Dmax;
    h2d(c, u, uniforms, sizeof(double) * S * L);
    mps_sample_core(psi, S, u, cfg, V0, V1, T, flag);
    double* hflag = pinned(c, 64);
    d2h(c, hflag, flag, 2);
    HIP_CHECK(hipMemcpyAsync(configs, cfg, sizeof(int) * S * L, hipMemcpyDeviceToHost, c->stream));
    sync(c);
    sample_flags(hflag[0], hflag[1]);
}

void mps_sample_noalloc(ite_mps* psi, int S, const double* u_dev, int* cfg_dev, double* scratch, size_t scratch_doubles) {
    ite_ctx* c = psi->ctx;
    const int L = psi->L;
    ITE_REQUIRE(S >= 1, "mps_sample_noalloc: nsamples must be >= 1");
    const size_t nw = mps_sample_scratch_doubles(psi, S);
    if (nw > scratch_doubles)
        ITE_FAIL(ITE_EINVAL, "mps_sample_noalloc: nsamples * (2 + d_max) * D_max * 8 + 256 = " +
                                 std::to_string(nw * 8) + " bytes exceeds the fixed scratch of " +
                                 std::to_string(scratch_doubles * 8) + " bytes");
    int Dmax = 1;
    for (int i = 0; i < L; ++i) Dmax = std::max(Dmax, psi->D[i + 1]);
    double* V0 = scratch + 32;
    double* V1 = V0 + (size_t)S * Dmax;
    double* T = V1 + (size_t)S * Dmax;
    mps_sample_core(psi, S, u_dev, cfg_dev, V0, V1, T, scratch);
    double hflag[2] = {0.0, 0.0};
    HIP_CHECK(hipMemcpyAsync(hflag, scratch, sizeof(hflag), hipMemcpyDeviceToHost, c->stream));
    sync(c);
    sample_flags(hflag[0], hflag[1]);
}

}  // namespace ite
