// Host-side objects of the library: context, MPO and MPS handles, and the
// operations of one implicit step (effective-Hamiltonian product,
// environment updates, GMRES local solve, Jacobi split, sweep).
#pragma once

#include "internal.h"

#include <array>
#include <string>
#include <vector>

// Workspace slots of a context (grow-only device buffers).
enum SlotId {
    SL_X1, SL_X3,                  // contraction intermediates
    SL_TPSI, SL_B, SL_TH,          // theta_psi, right-hand side, solution
    SL_V, SL_W,                    // Krylov basis, work vector
    SL_PART, SL_SMALL,             // reduction partials, small device scalars
    SL_Z, SL_GRAM, SL_ROT, SL_OFF, SL_NORM, SL_PERM,   // Jacobi split
    SL_QR,                         // Householder preconditioning
    SL_TMPA, SL_TMPB,              // scratch environments (overlap, energy)
    SL_LO_L, SL_LO_R, SL_LO_T, SL_LO_X,   // low-precision shadows (mixed precision)
    SL_R64, SL_D64,                // refinement residual and correction
    SL_HESS,                       // Hessenberg columns of a fixed-budget GMRES cycle
    SL_STATS,                      // per-block device records of the local solves of a step
    SL_BATCH, SL_BDESC, SL_BATCHB, // batched solves: workspaces, descriptors, per-state b and guess
    SL_TUNE,                       // tile autotuner: trial output
    SL_DMF, SL_DM1, SL_DM2, SL_DM3, SL_DMC,   // density-matrix MPO-MPS product: environments,
    SL_DMR, SL_DMV, SL_DMU,                   // intermediates, kept part, density matrix and its split
    SL_SPLITK,                     // K parts of under-filled FP64 products
    SL_NSLOTS
};

struct ite_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    ite_allocator alloc{};
    bool has_alloc = false;
    std::string err;
    void* slot_ptr[SL_NSLOTS] = {};
    size_t slot_bytes[SL_NSLOTS] = {};
    double* pinned = nullptr;      // host staging (hipHostMalloc)
    size_t pinned_bytes = 0;
    std::vector<hipEvent_t> events;
    size_t events_used = 0;
    // launch profiler (observability): FP64 GEMM launches are all timed,
    // Jacobi launches every `jac_period`-th of a kind; see LaunchProbe
    bool prof_on = false;
    int jac_period = 32;
    std::vector<hipEvent_t> prof_events;
    size_t prof_used = 0;
    std::vector<int> prof_kind;                 // kind of each recorded event pair
    long long prof_launches[ite::PK_COUNT] = {};
    long long prof_timed[ite::PK_COUNT] = {};
    double prof_ms[ite::PK_COUNT] = {};
    double prof_flops[ite::PK_COUNT] = {}, prof_bytes[ite::PK_COUNT] = {};
    // batched solves: a private stream (ordered after `stream` by events) on
    // which the launch sequence of a batch is captured as a graph and
    // replayed while the batch keeps its size, budget and precision
    bool use_graphs = true;
    hipStream_t side = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    // captured batched solves, keyed by (batch size, Krylov dimension and
    // precision, cycles, descriptor address, layout bytes); least recently
    // used first, at most BGRAPH_CACHE
    struct BatchGraph {
        long long key[5];
        hipGraphExec_t exec;
    };
    std::vector<BatchGraph> bgraphs;
    long long graph_captures = 0, graph_replays = 0, batch_solves = 0;
    long long graph_fallbacks = 0;   // batched solves issued directly after a capture was invalidated
    std::vector<char> batch_host;   // host image of the batch descriptors (kept until the next batch)
    int gemm_slots = 0;             // concurrent GEMM workgroups (two per compute unit), queried once
};

// Sparse small matrix in CSR form on the device.
struct CsrDev {
    int I = 0, O = 0, nnz = 0;
    int* rowptr = nullptr;
    int* col = nullptr;
    double* val = nullptr;
};

struct ite_mpo {
    ite_ctx* ctx = nullptr;
    int L = 0;
    std::vector<int> d, w;
    std::vector<std::vector<double>> Wh;   // host copies [wl][wr][out][in]
    std::vector<CsrDev> pair;   // two-site product W_j W_(j+1): (w_j, s, t) -> (p, q, w_(j+2))
    std::vector<CsrDev> left;   // (w_j, s) -> (p, w_(j+1))
    std::vector<CsrDev> right;  // (w_(j+1), s) -> (p, w_j)
    std::vector<CsrDev> ident;  // identity of size d (index by d)
    void* block = nullptr;      // one device allocation holding every CSR array
};

// Environments of one bond.
struct BondEnv {
    double* H = nullptr;    // <x|H|x>   [Dx][w][Dx]
    double* Hp = nullptr;   // <x|H|psi> [Dx][w][Dpsi]
    double* O = nullptr;    // <x|psi>   [Dx][Dpsi]
    bool hp_alias = false;  // Hp equals H (x = psi on this side)
    bool o_ident = false;   // O is the identity (x = psi on this side)
};

struct ite_mps {
    ite_ctx* ctx = nullptr;
    int L = 0;
    int chi_max = 1;
    std::vector<int> d;
    std::vector<int> D;      // current bond dimensions (L + 1)
    std::vector<int> Dcap;   // capacity of each bond
    std::vector<double*> A;  // site tensors
    double tau = 0.0;
    bool e_valid = false;
    double energy = 0.0;
    // evolution storage (allocated on the first step)
    std::vector<double*> X;      // working copy x
    std::vector<int> XD;         // bond dimensions of x
    std::vector<BondEnv> env;
    int env_w = 0;               // MPO bond dimension the environments were sized for
    // auxiliary state of the panel and MPS right-hand-side steps (the
    // augmented node-site state, or b), kept between steps; owned
    ite_mps* aux = nullptr;
};

namespace ite {

void* dev_alloc(ite_ctx* c, size_t bytes);
void dev_free(ite_ctx* c, void* p);
void* slot(ite_ctx* c, SlotId s, size_t bytes);
template <typename T> inline T* slot_t(ite_ctx* c, SlotId s, size_t count) {
    return static_cast<T*>(slot(c, s, count * sizeof(T)));
}
double* pinned(ite_ctx* c, size_t doubles);
void sync(ite_ctx* c);
void prof_collect(ite_ctx* c);

// Contraction primitives (device pointers; MPO matrices from ite_mpo).
struct HeffShape {
    int Dxl, Dyl, Dxr, Dyr, d1, d2, w0, w2;
};
// y = beta * H_eff theta + alpha * Cadd (Cadd may be null; y may alias Cadd).
// prec F32 / BF16: operands rounded to that precision (Llo / Rlo: environments
// already rounded, else rounded here), FP32 accumulation, FP64 output.
// FP32 / BF16 copies of the environments of a low-precision product (context
// buffers, valid until the next call), as a local solve makes them once.
void lo_shadows(ite_ctx* c, const HeffShape& s, Prec prec, const double* L, const double* R, const void** Llo,
                const void** Rlo);
void heff_apply(ite_ctx* c, const HeffShape& s, const double* L, const CsrDev& ww, const double* R,
                const double* theta, double beta, double alpha, const double* Cadd, double* y,
                Prec prec, const void* Llo = nullptr, const void* Rlo = nullptr);
// y = alpha * Lo theta Ro^T with Lo [Dxl][Dyl], Ro [Dxr][Dyr] (null = identity)
void overlap_apply(ite_ctx* c, int Dxl, int Dyl, int Dxr, int Dyr, int d1, int d2, const double* Lo,
                   const double* Ro, const double* theta, double alpha, double* y);
// Environment updates; W null = overlap environment.
void env_left(ite_ctx* c, int Dxa, int Dya, int Dxb, int Dyb, int d, int wl, int wr, const double* E,
              const double* X, const CsrDev* W, const double* Y, double* Eout);
void env_right(ite_ctx* c, int Dxa, int Dya, int Dxb, int Dyb, int d, int wl, int wr, const double* E,
               const double* X, const CsrDev* W, const double* Y, double* Eout);
// Overlap environment from the right: E'[b', b] = sum E[c', c] X[b', s, c'] Y[b, s, c]
// (ident: identity CSR of size d, used for the index permutation).
void env_right_overlap_pub(ite_ctx* c, const CsrDev& ident, int Dxa, int Dya, int Dxb, int Dyb, int d,
                           const double* E, const double* X, const double* Y, double* Eout);
// C = A1 A2 for site tensors A1 [Dl][d1][Dm], A2 [Dm][d2][Dr]
void two_site(ite_ctx* c, int Dl, int d1, int Dm, int d2, int Dr, const double* A1, const double* A2,
              double* theta);

struct SplitResult {
    int k = 0;
    double disc = 0.0;
    int sweeps = 0;
};
SplitResult split(ite_ctx* c, int dir, int Dl, int d1, int d2, int Dr, const double* theta, int chi_max,
                  double cutoff, double tie_rel, double* A1, double* A2, std::vector<double>* sigma);
// Truncation rule on sigma sorted descending (host).
int truncation_rank(const std::vector<double>& s, double cutoff, int chi_max, double tie_rel);

struct SolveStats {
    int matvecs64 = 0, matvecs_lo = 0;
    double res_rel = 0.0;
    int flags = 0;
    bool deferred = false;   // the figures are in the caller's device record, not here
};
// Linear operator of a local solve: y = alpha v + beta H_eff v.
struct LocalOp {
    HeffShape s;
    const double* L;
    const double* R;
    const CsrDev* ww;
    double alpha, beta;
    // low-precision products: environments rounded once per local solve
    Prec prec = Prec::F64;
    const void* Llo = nullptr;
    const void* Rlo = nullptr;
    size_t n() const { return (size_t)s.Dxl * s.d1 * s.d2 * s.Dxr; }
};
// stats_dev (nullable): device record of 8 doubles; with it, a solve with the
// fixed budget in FP64 runs without waiting for the host and leaves its
// figures there (SolveStats::deferred; [0] residual, [1] products, [2] flags).
SolveStats local_solve(ite_ctx* c, const LocalOp& op, const double* b, double* x, int m, int max_cycles,
                       double tol, int precision, int max_refine, double tol_refine, double* stats_dev = nullptr);

// One local solve of a batch: the operator, the right-hand side, the
// solution (initial guess on entry) and the device record of its figures.
struct BatchItem {
    LocalOp op;
    const double* b;
    double* x;
    double* stats;
};
// Fixed-budget FP64 GMRES(m) of every item at once (grouped products and
// batched vector kernels, captured as a graph when the context allows):
// item by item the same arithmetic as local_solve with a device record.
// Every item needs m < n, m <= 16 and at most 128 MPO-stage inputs.  lo:
// FP32 refinement, max_cycles corrections of one cycle each (the Arnoldi
// products with FP32 operands; the residual product and the basis FP64).
void gmres_batch(ite_ctx* c, const std::vector<BatchItem>& items, int m, int max_cycles, bool lo = false);
// Tile size (128 or 64) the autotuner picked for an FP64 GEMM shape.
int tuned_tile(ite_ctx* c, const Gemm& g);
// One implicit step of every state (ite_step_batch); status[j] gets each
// state's status (a failed state is left unchanged).
void step_batch(int n, ite_mps* const* psi, const ite_mpo* const* H, const double* h,
                const ite_step_opts* const* opts, ite_step_report* reps, int* status);

double dot(ite_ctx* c, const double* x, const double* y, size_t n);

// Copies on the context's stream (asynchronous) and the FP64 GEMM / sparse
// MPO stage on it (profiled like every contraction of the step).
void d2h(ite_ctx* c, double* host, const double* dev, size_t n);
void h2d(ite_ctx* c, void* dev, const void* host, size_t bytes);
// Blocking copies through the context's stream.
void h2d_wait(ite_ctx* c, void* dev, const void* host, size_t bytes);
void d2h_wait(ite_ctx* c, void* host, const void* dev, size_t bytes);
void d2d(ite_ctx* c, double* dst, const double* src, size_t n);
void gemm(ite_ctx* c, bool tA, bool tB, int M, int N, int K, double alpha, const double* A, long lda,
          const double* B, long ldb, double beta, const double* C, long ldc, double* D, long ldd);
void stage(ite_ctx* c, const CsrDev& m, Stage st);

// Sparse matrices of the MPO stages: a dense O x I matrix in CSR form, and
// the upload of several into one device allocation (*block, freed by the
// caller with dev_free).
struct CsrHost {
    int I = 0, O = 0;
    std::vector<int> rowptr, col;
    std::vector<double> val;
};
CsrHost dense_to_csr(const std::vector<double>& M, int O, int I);
std::vector<CsrDev> upload_csr(ite_ctx* c, const std::vector<CsrHost>& hs, void** block);

// Handles
ite_mpo* mpo_load(ite_ctx* c, int L, const int* d, const int* w, const double* const* W);
void mpo_destroy(ite_mpo* m);
ite_mps* mps_new(ite_ctx* c, int L, const int* d, int chi_max);
void mps_destroy(ite_mps* p);
// One step by the options' scheme (panel.cpp dispatches): the Gauss-Legendre
// panel and the MPS right-hand side are built on imag_step_sweep, the plain
// two-site sweep of one implicit step.
void imag_step(ite_mps* psi, const ite_mpo* H, double h, const ite_step_opts& o, ite_step_report* rep);
void imag_step_sweep(ite_mps* psi, const ite_mpo* H, double h, const ite_step_opts& o, ite_step_report* rep);
// Steps the lockstep batch cannot take (panel and MPS right-hand side).
bool step_is_composite(const ite_step_opts& o);
// Validation of step options (EINVAL with the reason).
void check_step(const ite_mps* psi, const ite_mpo* H, double h, const ite_step_opts& o);
// Bond capacities min(prod d left, prod d right, chi_max).
std::vector<int> bond_caps(int L, const std::vector<int>& d, int chi_max);
// Coefficients of a p-node Gauss-Legendre collocation panel: nodes c and
// weights b on [0, 1], A (p x p, row-major, A_ij = int_0^(c_i) l_j), the end
// weights w = A^-T b and r_inf = 1 - b^T A^-1 1.
struct GlCoef {
    int p = 0;
    std::vector<double> c, b, A, w;
    double r_inf = 0.0;
};
GlCoef gl_coefficients(int p);
// Density-matrix MPO-MPS product out = O psi (see ite_mpo_apply); out has
// psi's L, d and chi_max.  Returns the largest discarded-weight fraction.
double mpo_apply_dm(ite_mps* psi, const ite_mpo* O, int chi_max, double cutoff, double tie_rel, ite_mps* out);
double measure_energy(ite_mps* psi, const ite_mpo* H);
double overlap(ite_mps* a, ite_mps* b);

// Two-site DMRG ground-state sweeps (local problems: lowest eigenpair by
// Lanczos); see ite_dmrg_sweeps.
struct DmrgOpts {
    int nsweeps = 1, chi_max = 1, krylov_dim = 10, max_cycles = 1;
    double cutoff = 0.0, tie_rel = 1e-10, tol = 0.0;
};
struct DmrgReport {
    double energy = 0.0, max_res_rel = 0.0, max_disc = 0.0;
    long long matvecs = 0;
    int max_chi = 0;
};
void dmrg_sweeps(ite_mps* psi, const ite_mpo* H, const DmrgOpts& o, DmrgReport* rep);
// <psi|O_site|psi> / <psi|psi> for a one-site operator op_host [d][d] (host,
// (out, in)); psi right-orthonormal right of the site.
double site_expect(ite_mps* psi, int site, const double* op_host);
// Product-basis samples of psi (see ite_mps_sample); host arrays.
void mps_sample(ite_mps* psi, int nsamples, const double* uniforms, int* configs);
// Doubles of working memory mps_sample needs for nsamples samples of psi.
size_t mps_sample_scratch_doubles(const ite_mps* psi, int nsamples);
// The same samples from device uniforms into device configs, with the working
// vectors in the caller-given scratch (scratch_doubles long): no allocation.
void mps_sample_noalloc(ite_mps* psi, int nsamples, const double* u_dev, int* cfg_dev, double* scratch,
                        size_t scratch_doubles);
// Fixed per-device scratch of the no-allocation entry point (noalloc.hip).
void noalloc_init(int device);
double* noalloc_scratch(int device);
size_t noalloc_scratch_doubles();

}  // namespace ite
