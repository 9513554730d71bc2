/*
 * ite.h -- C ABI of the MI355X (gfx950) implicit imaginary-time evolution
 * library for matrix product states.
 *
 * The library advances an MPS |psi> under an MPO Hamiltonian H by A-stable
 * implicit steps on logarithmic tau grids, following "Fast Tensor Network
 * Imaginary Time Evolution by Implicit Stepping on Logarithmic Grids"
 * (Zima, Stoudenmire, White, Parcollet, Kaye):
 *
 *   trapezoid rule (Method, Eq. 4):  (I + h (H - s)) x = (I - h (H - s)) psi,
 *                                    h = dtau / 2;
 *   backward Euler:                  (I + h (H - s)) x = psi, h = dtau;
 *
 * solved in MPS form by a two-site DMRG-style sweep whose local problems are
 * GMRES solves with the effective Hamiltonian (Method, last paragraph;
 * Appendix B), followed by normalisation and, optionally, a shift s equal to
 * the energy of the current state (Appendix D).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Numbers on the boundary are real FP64.  Arrays are row-major, last
 *    index fastest.  Site tensors A_i[D_(i-1)][d_i][D_i]; MPO tensors
 *    W_i[w_i][w_(i+1)][d_i (out)][d_i (in)] with w_0 = w_L = 1.
 *  - Host arrays passed in are copied before the call returns; the caller
 *    keeps ownership.  Outputs go to caller-allocated host memory.
 *  - Device memory is owned by the context and obtained from the caller's
 *    allocator (or hipMalloc when none is given).  Handles own their device
 *    tensors until *_destroy.
 *  - All device work of a context is ordered on the HIP stream given at
 *    creation.  Calls return after their work has finished (synchronous at
 *    step granularity).  A context is not thread-safe: one context per host
 *    thread.
 *  - Every function returns an int status (ITE_OK = 0 or a negative code).
 *    No C++ exception crosses the ABI.  ite_last_error() gives the text of
 *    the last failure on a context.
 */
#ifndef ITE_H
#define ITE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define ITE_OK          0
#define ITE_EINVAL     (-1)   /* invalid argument (shape, range, non-finite input) */
#define ITE_ENOMEM     (-2)   /* allocator returned NULL, or an admission cap was exceeded */
#define ITE_EDEVICE    (-3)   /* a HIP call failed; see ite_last_error */
#define ITE_ESTATE     (-4)   /* objects do not fit together (e.g. MPS and MPO of different L) */
#define ITE_ENONFINITE (-5)   /* the step produced a non-finite state; psi was left unchanged */

/* ---- enumerations ------------------------------------------------------ */
enum { ITE_SCHEME_TRAP = 0, ITE_SCHEME_BE = 1, ITE_SCHEME_GL = 2 };
enum { ITE_SHIFT_FIXED = 0, ITE_SHIFT_TRACK = 1 };
enum { ITE_PREC_FP64 = 0, ITE_PREC_FP32_IR = 1, ITE_PREC_BF16_IR = 2 };
enum { ITE_GUESS_PSI = 0, ITE_GUESS_B = 1 };
enum { ITE_RHS_PROJECT = 0, ITE_RHS_MPS = 1 };

/* report flags */
#define ITE_FLAG_BUDGET_EXHAUSTED 1  /* a local solve ended on its Krylov budget above tol_loc (normal in budget mode) */
#define ITE_FLAG_BREAKDOWN        2  /* an Arnoldi step found an invariant subspace (exact local solve) */
#define ITE_FLAG_REFINE_LIMIT     4  /* mixed precision: refinement stopped at max_refine above tol_refine */

/* ---- opaque handles ---------------------------------------------------- */
typedef struct ite_ctx ite_ctx;
typedef struct ite_mpo ite_mpo;
typedef struct ite_mps ite_mps;
typedef struct ite_server ite_server;

/* Device allocator supplied by the caller (e.g. a framework's caching
 * allocator).  alloc returns device memory of at least `bytes` bytes usable on
 * the context's stream, or NULL; free releases it.  Both are called from the
 * thread that calls the library. */
typedef struct ite_allocator {
    void* (*alloc)(size_t bytes, void* user);
    void  (*free)(void* ptr, void* user);
    void* user;
} ite_allocator;

/* Options of one implicit step.  ite_default_opts() fills the paper's budget:
 * trapezoid, shift tracking, Krylov dimension 10, one GMRES cycle, one sweep
 * (Appendix D), cutoff 1e-10 (Heisenberg chain section), the right-hand side as
 * the first local solve's initial guess (Appendix B); FP64 products, and
 * for the mixed precisions max_refine 0 (one correction for FP32-IR, which
 * spends the same single GMRES cycle on the FP64 residual of x0, two for
 * BF16-IR) with tol_refine 0. */
typedef struct ite_step_opts {
    int    scheme;       /* ITE_SCHEME_TRAP or ITE_SCHEME_BE */
    int    shift_mode;   /* ITE_SHIFT_FIXED (use `shift`) or ITE_SHIFT_TRACK (s = energy of psi) */
    double shift;
    int    chi_max;      /* bond dimension cap, >= 1 */
    double cutoff;       /* discarded-weight fraction; 0 keeps min(rows, cols, chi_max) values */
    double tie_rel;      /* a cut inside a group of values closer than tie_rel*sigma_0 moves below it */
    int    krylov_dim;   /* Arnoldi steps per GMRES cycle, 1..64 */
    int    max_cycles;   /* GMRES cycles per local solve, >= 1 */
    double tol_loc;      /* relative residual target; 0 = fixed budget (no early exit) */
    int    nsweeps;      /* full (left-right-left) sweeps per step, >= 1 */
    int    precision;    /* ITE_PREC_*: inner matvec precision of the local solves */
    int    max_refine;   /* mixed precision: refinement rounds (corrections) per local solve;
                          * 0 = the cheapest count that keeps the fixed-budget step within
                          * 1e-8 relative energy of the FP64 step: 1 for FP32-IR, 2 for
                          * BF16-IR */
    double tol_refine;   /* mixed precision: FP64 relative residual target; 0: exactly max_refine
                          * corrections, no FP64 residual after the last one (the reported
                          * residual is then the inner GMRES estimate) */
    int    init_guess;   /* ITE_GUESS_B: the step's first local solve starts from b projected
                          * into x's basis (Appendix B uses the right-hand side as the initial
                          * guess), later ones from the current x_j x_(j+1); ITE_GUESS_PSI:
                          * x_j x_(j+1) throughout.  Identical for backward Euler (b = psi). */
    int    gl_nodes;     /* ITE_SCHEME_GL: Gauss-Legendre nodes p per panel, 1..7 (default 2) */
    int    rhs_mode;     /* trapezoid right-hand side: ITE_RHS_PROJECT (default) projects
                          * (I - h (H - s)) psi into x's basis exactly through mixed environments;
                          * ITE_RHS_MPS first forms it as an MPS b by the density-matrix MPO-MPS
                          * product (Appendix B; truncated by chi_max / cutoff / tie_rel like a
                          * split) and solves with b in place of psi, x starting as b */
} ite_step_opts;

/* Per-step report. */
typedef struct ite_step_report {
    double tau;          /* tau after the step */
    double dtau;         /* step length (2h for the trapezoid rule, h for backward Euler) */
    double h;
    double shift;
    double energy;       /* <psi|H|psi> of the normalised new state */
    double norm_before;  /* ||x|| before renormalisation */
    int    max_chi;
    int    flags;        /* ITE_FLAG_* */
    double max_disc;     /* largest discarded-weight fraction over the splits */
    double sum_disc;
    double max_res_rel;  /* largest local relative residual estimate */
    double mean_res_rel;
    long long matvecs_fp64;  /* effective-Hamiltonian products in FP64 */
    long long matvecs_lo;    /* ... in FP32 or BF16 */
    double ms_total, ms_rhs, ms_solve, ms_split, ms_env;   /* device time per phase (the density-matrix
                          * product of ITE_RHS_MPS counts as rhs, a panel's read-off and cut-back as
                          * split; those two are timed on the host around a drained stream) */
    double rhs_disc;     /* ITE_RHS_MPS: largest discarded-weight fraction of the density-matrix product */
    int    aux_max_chi;  /* ITE_SCHEME_GL: largest bond of the augmented (node-site) state before it
                          * is cut back to the chain's bonds */
} ite_step_report;

/* ---- context ----------------------------------------------------------- */

/* Create a context on HIP device `device`.  hip_stream: a hipStream_t (NULL =
 * the default stream).  alloc: NULL for hipMalloc/hipFree.  Errors: EINVAL
 * (bad device or NULL out), EDEVICE. */
int ite_ctx_create(int device, void* hip_stream, const ite_allocator* alloc, ite_ctx** out);
int ite_ctx_destroy(ite_ctx* ctx);
/* Text of the last error on ctx (never NULL; empty when none).  Valid until
 * the next call on ctx. */
const char* ite_last_error(const ite_ctx* ctx);
/* Library version string. */
const char* ite_version(void);

/* Launch profiler (observability, used by the benchmark): with enable = 1
 * the context brackets FP64 contraction launches (all) and Jacobi launches
 * (a sample) with HIP events on its stream and counts their algorithmic work;
 * enabling resets the totals, enable = 0 stops recording.
 * ite_ctx_profile_read synchronises the stream and returns, for the FP64
 * contraction GEMMs, the launch count, the summed device time (ms) and the
 * summed algorithmic flops 2 M N K since the last enable. */
int ite_ctx_profile(ite_ctx* ctx, int enable);
int ite_ctx_profile_read(ite_ctx* ctx, long long* launches, double* ms, double* flops);
/* Per-kernel launch profile since the last enable, by kind: 0 FP64
 * contraction GEMMs (every launch timed), 1 Jacobi Gram, 2 Jacobi inner
 * sweep, 3 Jacobi rotation (every 32nd launch of a kind timed).  launches: all
 * launches; timed, ms_timed: the timed ones and their summed device time;
 * flops, bytes: the algorithmic work of all launches (Jacobi: of the pairs
 * and column chunks the kernels actually processed). */
int ite_ctx_profile_kernel(ite_ctx* ctx, int kind, long long* launches, long long* timed,
                           double* ms_timed, double* flops, double* bytes);

/* Fill `o` with the defaults described at ite_step_opts. */
void ite_default_opts(ite_step_opts* o);

/* ---- Hamiltonian ------------------------------------------------------- */

/* Load an MPO (Method: the Hamiltonian is represented as an MPO; Appendix B:
 * the Heisenberg and impurity MPOs are exact sums of local terms with modest
 * bond dimension).  d[L] local dimensions, w[L+1] MPO bond dimensions with
 * w[0] = w[L] = 1, W[i] points to w[i]*w[i+1]*d[i]*d[i] doubles in
 * [wl][wr][out][in] order (host memory).  Every MPO within these limits runs
 * (the two-site stage has at most 16 * 8 * 8 = 1024 inputs per column).
 * Errors: EINVAL (L < 2, d < 1, w[0] != 1, w[L] != 1, w > 16, d > 8,
 * non-finite entries, NULL pointers), ENOMEM, EDEVICE. */
int ite_mpo_load(ite_ctx* ctx, int L, const int* d, const int* w,
                 const double* const* W, ite_mpo** out);
int ite_mpo_destroy(ite_mpo* mpo);

/* ---- states ------------------------------------------------------------ */

/* Product state (the initial states of the paper are product states: the
 * Neel state of the Heisenberg chain section, the METTS product states of
 * Appendix D) from L normalised real spinors (spinors[i] has d[i] entries,
 * host memory; each is normalised again on entry).  chi_max bounds every
 * bond of the state for its lifetime.  pad_full = 0: all bonds have dimension
 * 1.  pad_full = 1: the state is embedded in bonds of dimension
 * D_i = min(d_1..d_i, d_(i+1)..d_L, chi_max) (products of local dimensions):
 * row 0 of site i (as a D_(i-1) x (d_i D_i) matrix) is spinor_i (x) e_0 and
 * the other rows are the remaining rows of the Householder reflector that maps
 * e_0 to it, so the tensors are right-orthonormal and the state is unchanged.
 * Errors: EINVAL (L < 2, chi_max < 1, zero or non-finite spinor), ENOMEM,
 * EDEVICE. */
int ite_mps_create(ite_ctx* ctx, int L, const int* d, const double* const* spinors,
                   int chi_max, int pad_full, ite_mps** out);

/* Load an MPS (Method: the state is represented as an MPS) from site tensors
 * (host memory, A[i] has chi[i]*d[i]*chi[i+1] doubles).  The
 * tensors must be right-orthonormal (each A_i as a chi[i] x (d_i chi[i+1])
 * matrix has orthonormal rows for i >= 2) with the norm on site 1 -- the form
 * every step leaves behind; this is not checked beyond finiteness.  chi[0] =
 * chi[L] = 1, chi[i] <= chi_max.  Used for checkpoints and tests. */
int ite_mps_load(ite_ctx* ctx, int L, const int* d, const int* chi,
                 const double* const* A, int chi_max, ite_mps** out);

/* Export the MPS (Method: the state as an MPS) -- bond dimensions (chi[L+1],
 * required) and, when A is not NULL, the site tensors into caller buffers A[i]
 * of at least chi[i]*d[i]*chi[i+1] doubles (call first with A = NULL to learn
 * the sizes).  Right-orthonormal with the norm on site 1.  Errors: EINVAL
 * (NULL psi or chi), EDEVICE. */
int ite_mps_export(ite_mps* psi, int* chi, double* const* A);
int ite_mps_destroy(ite_mps* psi);

/* Imaginary time carried by the state (advanced by every step, set to 0 at
 * creation); ite_mps_set_tau changes it (checkpoint resume). */
int ite_mps_get_tau(const ite_mps* psi, double* tau);
int ite_mps_set_tau(ite_mps* psi, double tau);

/* ---- the method ---------------------------------------------------------- */

/* One implicit step (Method, Eq. 4; Appendix B; Appendix D):
 * solve (I + h (H - s)) x = b with b = psi (BE) or (I - h (H - s)) psi (TRAP)
 * by one or more two-site sweeps of GMRES local solves with SVD truncation,
 * normalise, and replace psi by x.  s is opts->shift (FIXED) or <psi|H|psi>
 * (TRACK).  tau advances by h (BE) or 2h (TRAP).  rep may be NULL.
 * With opts->rhs_mode = ITE_RHS_MPS the trapezoid right-hand side is first
 * formed as an MPS by the density-matrix product (ite_mpo_apply of the MPO
 * of (1 + h s) I - h H, truncated by chi_max, cutoff, tie_rel; Appendix B),
 * and the solve runs as the backward-Euler form with that MPS in place of
 * psi (x starts as b; rep->rhs_disc reports the product's truncation).
 * ITE_SCHEME_GL (Method: the spectral variant) advances psi over one panel
 * of length h by p = opts->gl_nodes point Gauss-Legendre collocation: the
 * node values Y_1..Y_p of the polynomial solution satisfy the integral form
 * of the evolution equation (Eq. 2 from the panel's start) at the nodes,
 * (I + h A (x) (H - s)) Y = 1 (x) psi with A_ij the integral of the j-th
 * Lagrange polynomial from 0 to node c_i.  The p node values are one MPS on
 * L + 1 sites whose first site (dimension p + 1, entry 0 = psi itself)
 * indexes the node, so the system is one backward-Euler-type solve of the
 * augmented MPO (the node matrix [[0, 0], [0, A]] times the MPO of H - s)
 * by the same sweep; the panel's end value r_inf psi + sum_j w_j Y_j (the
 * (p, p) Pade approximant of exp(-h (H - s)) applied to psi; w = A^-T b for
 * the Gauss weights b, r_inf = 1 - b^T A^-1 1) is the node site contracted
 * into site 1, with the bonds cut back to the chain's own by exact two-site
 * splits; then normalised.  tau advances by h.  When p + 1 exceeds d_1 D_2
 * (the most rank the sweep's first block can give the node bond with psi's
 * bonds), the augmented state's bonds are first widened by zero-weight
 * orthonormal completions: to complete where that is within chi_max, else
 * to what the node rank needs to pass; so the sweep gives the panel exactly
 * at complete bonds for any p.
 * Errors: EINVAL (h <= 0 or non-finite, bad options), ESTATE (L or d of psi
 * and H differ), ENOMEM, EDEVICE, ENONFINITE (psi left unchanged). */
int ite_imag_step(ite_mps* psi, const ite_mpo* H, double h,
                  const ite_step_opts* opts, ite_step_report* rep);

/* One implicit step (as ite_imag_step) of each of n independent states, run
 * as a batch: the sweeps advance in lockstep block by block, and the
 * fixed-budget GMRES local solves of a block slot run together -- one
 * grouped launch per contraction stage for the H_eff products of all states
 * (uneven bond dimensions, tile size per GEMM shape from the library's
 * autotuner), one batched launch per Krylov vector operation, the small
 * least-squares solves on the device -- captured as a HIP graph on a
 * private stream (ordered after ctx's stream) and replayed while the batch
 * keeps its size, budget and precision (the last four such graphs are kept;
 * a capture that another thread's call invalidates is issued directly).
 * FP64 solves and FP32 refinement with a fixed number of corrections
 * (tol_refine = 0, max_cycles = 1: one cycle per correction, the Arnoldi
 * products FP32) batch, each precision in its own group.  Serving
 * (Appendix D: many independent METTS evolutions) advances its active
 * requests this way.  Every state must be on ctx; h[j] and opts[j] are state
 * j's; reps (nullable) gets n reports, status (nullable) each state's status
 * (a failed state is left unchanged).  Local solves outside the batched kind
 * (tolerance-driven, BF16 or tolerance-driven refinement, Krylov dimension
 * above 16 or not below the block's length, more than 128 MPO-stage inputs)
 * run one by one within the same slots.  A state's result is bitwise the
 * same in any batch, alone included, and equals ite_imag_step's to rounding.  Returns OK, or the first failing state's status, or EINVAL /
 * ESTATE for bad arguments (nothing run). */
int ite_step_batch(ite_ctx* ctx, int n, ite_mps* const* psi, const ite_mpo* const* H, const double* h,
                   const ite_step_opts* const* opts, ite_step_report* reps, int* status);
/* Batched solves: enable (1, default) or disable (0) the graph capture (the
 * launches are then issued one by one on ctx's stream), and the counts of
 * batched solves, graph captures and graph replays since creation. */
int ite_ctx_set_graphs(ite_ctx* ctx, int enable);
int ite_ctx_batch_stats(ite_ctx* ctx, long long* solves, long long* captures, long long* replays);

/* Two-site DMRG ground-state sweeps (the ground state of the impurity model
 * that seeds the METTS chains and gives the zero-temperature double
 * occupancy, Appendix D), on the same blocks, environments and SVD split as
 * ite_imag_step: per block the lowest eigenpair of the two-site effective
 * Hamiltonian by Lanczos (Arnoldi steps with classical Gram-Schmidt twice,
 * at most krylov_dim vectors per cycle, restarted from the Ritz vector for
 * at most max_cycles cycles, or until ||H x - theta x|| <= tol |theta|;
 * tol = 0: the full budget), then the split (chi_max capped by psi's own
 * maximum, cutoff and tie_rel as in ite_step_opts).  One sweep is a
 * left-to-right plus a right-to-left half sweep; psi (any normalised state
 * with the centre on site 1, as left by the constructors and ite_imag_step)
 * is replaced by the result, normalised, centre on site 1; its tau is
 * unchanged.  Outputs (each nullable): *energy = <psi|H|psi> of the result,
 * *max_res_rel the largest relative residual estimate of a local problem,
 * *max_disc the largest discarded weight, *matvecs the effective-Hamiltonian
 * products.  Errors: EINVAL (nsweeps or max_cycles < 1, krylov_dim outside
 * 1..64, chi_max < 1, cutoff outside [0, 1), tie_rel or tol < 0), ESTATE (L
 * or d of psi and H differ), ENOMEM, EDEVICE, ENONFINITE (psi left
 * unchanged). */
int ite_dmrg_sweeps(ite_mps* psi, const ite_mpo* H, int nsweeps, int chi_max, double cutoff,
                    double tie_rel, int krylov_dim, int max_cycles, double tol, double* energy,
                    double* max_res_rel, double* max_disc, long long* matvecs);

/* Product-basis samples of psi, the collapse step of a METTS chain
 * (Appendix D: a METTS |psi_i> is measured in a product basis, giving |j>
 * with probability |<j|psi_i>|^2; the chains start from product states
 * sampled from the ground state): site by site from the left, s_i drawn from
 * its conditional probability given s_1..s_(i-1), exact because psi is
 * right-orthonormal with the centre on site 1 (as every call of this library
 * leaves it; the norm cancels).  Sample k takes the first s with
 * P(s' <= s) > u and P(s) > 0, u = uniforms[i * nsamples + k] (host array,
 * L * nsamples values in [0, 1), drawn by the caller); configs (host,
 * nsamples * L ints) gets s_i of sample k at configs[k * L + i].  L must equal
 * psi's length: it states the size of both host buffers.
 * Errors: EINVAL (nsamples < 1, null arrays, L not psi's length, a uniform
 * outside [0, 1)), ENONFINITE (a conditional distribution with a zero or
 * non-finite total: psi is zero or not finite; configs are then meaningless),
 * ENOMEM, EDEVICE. */
int ite_mps_sample(ite_mps* psi, int nsamples, int L, const double* uniforms, int* configs);

/* <psi|O|psi> / <psi|psi> for a one-site operator O acting on `site`
 * (0-based), op[d_site][d_site] (host, row-major, (out, in)): the impurity
 * double occupancy n_(d,up) n_(d,dn) of Appendix D is diag(0, 0, 0, 1) on the
 * impurity site in the local basis |0>, |up>, |dn>, |up dn>.  psi must be
 * right-orthonormal right of the site (every state this library leaves is:
 * centre on site 1).  Errors: EINVAL (NULL pointers, site out of range,
 * non-finite entries, zero state), EDEVICE. */
int ite_mps_expect_site(ite_mps* psi, int site, const double* op, double* out);

/* A METTS chain (Appendix D): from the product state `start` (L local
 * indices; the paper seeds it with a sample of the ground state, e.g. from
 * ite_dmrg_sweeps and ite_mps_sample), nsamples times: |psi_k> ~
 * exp(-beta H / 2)|config_k> by ite_evolve_loggrid on the geometric grid
 * tau0 -> beta / 2 with `ratio` and `opts` (MPS created with chi_max, unit
 * bonds), the energy of |psi_k> (the last step's) into energies[k], <psi_k|O|psi_k>
 * for the one-site operator (site, op) as ite_mps_expect_site into
 * observables[k], config_k into configs[k * L .. k * L + L), then the
 * collapse to the next configuration by ite_mps_sample with the L uniforms
 * uniforms[k * L .. k * L + L) (host, in [0, 1)).  The thermal average of O is
 * the plain mean of observables.  The collapse in the computational basis
 * keeps every conserved quantity of the start state (particle number and S^z
 * for the impurity model), so the chain samples the canonical ensemble of the
 * start state's sector.  Host arrays; the chain runs on H's context.
 * Errors: EINVAL (NULL pointers, nsamples < 1, L not H's length, 0 < tau0 <
 * beta / 2 violated, ratio <= 1, site or start out of range), and those of
 * the calls it makes (the chain stops at the failing element). */
int ite_metts_chain(const ite_mpo* H, const int* start, int chi_max, double beta, double tau0, double ratio,
                    const ite_step_opts* opts, int site, const double* op, int nsamples, int L,
                    const double* uniforms, int* configs, double* energies, double* observables);

/* ite_mps_sample for callers that cannot allocate device or pinned host
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): the same samples, bit for bit, from DEVICE buffers --
 * uniforms (L * nsamples doubles, layout as ite_mps_sample) and configs
 * (nsamples * L ints) -- with every working vector in a fixed scratch array of
 * 64 MiB that the library reserves on each GPU it runs on until the process
 * ends.  The call allocates nothing; it needs
 * 256 + 8 * nsamples * (2 + d_max) * D_max bytes of that scratch (D_max the
 * largest bond of psi, d_max the largest local dimension), e.g. up to 2730
 * samples at D_max = 1024, d = 2.  Calls on one GPU share the array and keep
 * the last call's contents: calls that overlap in time on one GPU (from two
 * threads or two streams) race and give wrong samples.  Returns after configs
 * is written (synchronous on psi's stream).  Errors: EINVAL (NULL pointers,
 * nsamples < 1, L not psi's length, the scratch need above 64 MiB -- the
 * message states both sizes --, a uniform outside [0, 1)), ENONFINITE (as
 * ite_mps_sample), EDEVICE. */
int ite_mps_sample_noalloc(ite_mps* psi, int nsamples, int L, const double* uniforms, int* configs);

/* Evolve along the geometric grid 0, tau0, tau0 r, tau0 r^2, ... clamped to
 * end at tau1 (Method: logarithmic grids), starting at the first grid point
 * after psi's current tau.  per_step (nullable) receives up to max_steps
 * reports; *n_steps (nullable) the number of steps taken.  Errors: EINVAL
 * (tau0 <= 0, tau1 <= tau0, ratio <= 1, non-finite), plus those of
 * ite_imag_step (the evolution stops at the failing step). */
int ite_evolve_loggrid(ite_mps* psi, const ite_mpo* H, double tau0, double tau1, double ratio,
                       const ite_step_opts* opts, ite_step_report* per_step, int max_steps,
                       int* n_steps);

/* Evolve along an explicit increasing grid taus[0..n_taus) (e.g. the panel
 * grid of the Method section), starting at the first point after psi's tau. */
int ite_evolve_grid(ite_mps* psi, const ite_mpo* H, const double* taus, int n_taus,
                    const ite_step_opts* opts, ite_step_report* per_step, int max_steps,
                    int* n_steps);

/* phi = O psi by the "density matrix" algorithm for MPO-MPS products
 * (Appendix B applies the trapezoid right-hand side this way): left
 * environments F_j of <O psi|O psi> without truncation, then from the right
 * end, at each site, the tensor T_j of O_j psi_j contracted with what is
 * already kept to its right, its reduced density matrix rho_j = T^T F_j T
 * (over the site index and the kept right index), and the eigenvectors of
 * rho_j's largest eigenvalues (one-sided Jacobi, FP64) as the new
 * right-orthonormal site tensor; the kept count follows the split's rule
 * (cutoff, tie_rel) on the square roots of the eigenvalues, at most
 * min(chi_max, the bond's largest possible rank); site 1 keeps the rest
 * whole, so it holds the norm of phi.  O must have psi's L and local
 * dimensions and at most 128 MPO-index x local-dimension inputs per site.
 * *out receives a new MPS (same L, d and chi_max as psi, tau 0; destroy with
 * ite_mps_destroy); *max_disc (nullable) the largest discarded-weight
 * fraction.  psi is unchanged.  Errors: EINVAL (NULL pointers, chi_max < 1,
 * cutoff outside [0, 1), tie_rel < 0), ESTATE (shapes or contexts differ),
 * ENOMEM, EDEVICE, ENONFINITE (phi is zero or not finite; *out not set). */
int ite_mpo_apply(const ite_mpo* O, ite_mps* psi, int chi_max, double cutoff, double tie_rel,
                  ite_mps** out, double* max_disc);

/* Energy <psi|H|psi> / <psi|psi> (the quantity the trapezoid step's shift
 * tracks, Appendix D: the spectrum is shifted by the energy of the new state
 * each step; Method: the shift that puts the ground state energy at 0), by a
 * transfer contraction from the right with the MPO.  Also caches the value as
 * the shift of a following TRACK step.  Errors: EINVAL (NULL arguments),
 * ESTATE (different contexts or lengths), EDEVICE. */
int ite_measure_energy(ite_mps* psi, const ite_mpo* H, double* energy);
/* <a|b> by transfer matrices (the overlap of the Heisenberg chain section's
 * error measure, sqrt(1 - <psi|psi_ref>) for normalised states).  Same L and
 * local dimensions, same context; errors: EINVAL, ESTATE, EDEVICE. */
int ite_mps_overlap(ite_mps* a, ite_mps* b, double* out);
/* ||psi||, the norm of the centre tensor on site 1 (Appendix D: the state is
 * normalised after each step, so this is 1 after every step).  Errors:
 * EINVAL, EDEVICE. */
int ite_mps_norm(ite_mps* psi, double* out);

/* ---- grids (host only; no device work) ---------------------------------- */

/* Geometric grid of ite_evolve_loggrid: writes up to cap points (0 first) to
 * out and their number to *n.  EINVAL for bad parameters or cap too small
 * (then *n holds the required count). */
int ite_loggrid(double tau0, double tau1, double ratio, double* out, int cap, int* n);
/* Coefficients of a p-node Gauss-Legendre collocation panel (Method: the
 * spectral variant; the panel step of ITE_SCHEME_GL uses exactly these):
 * nodes c[p] (ascending) and weights b[p] on [0, 1], A[p*p] (row-major,
 * A_ij = integral from 0 to c_i of the Lagrange polynomial of node j), the
 * end weights w[p] = A^-T b and *r_inf = 1 - b^T A^-1 1.  Host only.
 * EINVAL for p outside 1..7 or NULL pointers. */
int ite_gl_coefficients(int p, double* c, double* b, double* A, double* w, double* r_inf);
/* Panel grid (Method): P panels with endpoints {0, tau_max / 2^(P-j)},
 * j = 1..P, and n uniform steps per panel: P*n + 1 points. */
int ite_panel_grid(double tau_max, int P, int n, double* out, int cap, int* npts);

/* ---- serving: many independent evolutions at once ----------------------
 * A request is one whole evolution as ite_evolve_loggrid runs it: a product
 * state (ite_mps_create), a Hamiltonian (ite_mpo_load), the geometric grid
 * tau0, tau1, ratio and the step options (Method; Appendix D for the
 * budget).  Requests are independent, as the METTS evolutions of the impurity
 * application are.  The server keeps `workers` host threads, each with its
 * own context on its own non-blocking HIP stream of device `device`, so the
 * steps of different requests run on the GPU at the same time.  Continuous
 * batching: a request waits in FIFO order until the summed footprint
 * estimate of the active requests plus its own fits `mem_cap` bytes and a
 * worker has fewer than `max_active` active requests; it then stays on that
 * worker, which advances all its active requests by one time step at a time as
 * one batch (ite_step_batch: grouped launches for their uneven-bond H_eff
 * products, a captured graph for the batched local solves), and leaves as
 * soon as its grid is done, making room for the next.  All device
 * memory comes from a pool owned by the server (no hipFree while the server
 * runs).  A request's arithmetic does not depend on what else is running:
 * its results are bitwise those of the same evolution run alone. */

typedef struct ite_server_opts {
    int    device;
    int    workers;      /* host threads = concurrent device streams, 1..64 */
    int    max_active;   /* active requests per worker, >= 1 */
    double mem_cap;      /* bytes; admission cap on the summed footprint estimates */
} ite_server_opts;

typedef struct ite_request {
    int L;
    const int* d;                    /* [L] local dimensions */
    const int* w;                    /* [L+1] MPO bond dimensions */
    const double* const* W;          /* [L] MPO tensors as ite_mpo_load (host) */
    const double* const* spinors;    /* [L] product state as ite_mps_create (host) */
    int chi_max;
    int pad_full;
    double tau0, tau1, ratio;        /* geometric grid as ite_evolve_loggrid */
    ite_step_opts opts;
} ite_request;

/* Request states */
#define ITE_REQ_PENDING  0
#define ITE_REQ_ACTIVE   1
#define ITE_REQ_DONE     2
#define ITE_REQ_FAILED   3

typedef struct ite_request_info {
    int status;          /* ITE_REQ_* */
    int error;           /* status code of the failure (ITE_REQ_FAILED) */
    int worker;          /* worker that ran it (-1 before admission) */
    int n_steps;         /* steps done so far */
    int n_grid;          /* steps of its grid */
    double tau, energy;  /* after the last step done */
    double footprint;    /* bytes, the admission estimate */
    double t_submit, t_admit, t_done;   /* seconds on the server clock (0 = not yet) */
} ite_request_info;

/* Create / destroy a server.  Destroy waits for the running steps, drops
 * pending requests and frees everything.  Errors: EINVAL, EDEVICE, ENOMEM. */
int ite_server_create(const ite_server_opts* o, ite_server** out);
int ite_server_destroy(ite_server* srv);
/* Queue a request (all arrays are copied before return) and return its id.
 * EINVAL for inconsistent inputs; ENOMEM when its footprint alone exceeds
 * mem_cap. */
int ite_server_submit(ite_server* srv, const ite_request* req, long long* id);
/* Wait until request `id` is DONE or FAILED, at most timeout_s seconds
 * (< 0: no limit); fills *info either way.  Returns OK when finished,
 * ESTATE on time-out, EINVAL for an unknown id. */
int ite_server_wait(ite_server* srv, long long id, double timeout_s, ite_request_info* info);
/* Current state of a request without waiting. */
int ite_server_info(ite_server* srv, long long id, ite_request_info* info);
/* Per-step reports of a finished request: up to cap reports to out, their
 * number to *n. */
int ite_server_reports(ite_server* srv, long long id, ite_step_report* out, int cap, int* n);
/* Final state of a finished request: bond dimensions to chi [L+1] and, when A
 * is not NULL, the site tensors to A[i] (host, chi[i] d[i] chi[i+1] each). */
int ite_server_state(ite_server* srv, long long id, int* chi, double* const* A);
/* Forget a finished request (its reports and state). */
int ite_server_release(ite_server* srv, long long id);
/* Server clock (seconds since creation) and the text of the last error of
 * a failed request (empty when none). */
double ite_server_clock(const ite_server* srv);
int ite_server_error(ite_server* srv, long long id, char* buf, int cap);
/* Footprint estimate (bytes) the server uses for admission: MPS and working
 * copy, environments, Krylov basis and the largest split workspace. */
double ite_request_footprint(int L, const int* d, const int* w, int chi_max, int krylov_dim);

/* ---- building blocks exposed for parity tests ---------------------------
 * Each operates on caller device memory on the context's stream and returns
 * after it has finished. */

/* D = alpha op(A) op(B) + beta C in FP64 (row-major; op = transpose when
 * trans* != 0; C may be NULL).  prec: ITE_PREC_FP64 (FP64 MFMA),
 * ITE_PREC_FP32_IR (operands rounded to FP32, FP32 MFMA, FP32 accumulation),
 * ITE_PREC_BF16_IR (operands rounded to BF16, BF16 MFMA, FP32 accumulation). */
int ite_debug_gemm(ite_ctx* ctx, int transA, int transB, int M, int N, int K, double alpha,
                   const double* A, int lda, const double* B, int ldb, double beta,
                   const double* C, int ldc, double* D, int ldd, int prec);

/* y = alpha theta + beta H_eff theta for the two-site effective Hamiltonian
 * (Method; Appendix B):
 *   H_eff theta [a', p, q, c'] = sum L[a', w, a] W1[w, v, p, s] W2[v, u, q, t]
 *                                    R[c', u, c] theta[a, s, t, c].
 * Shapes: L [Dxl][w0][Dyl], R [Dxr][w2][Dyr], W1 [w0][w1][d1][d1],
 * W2 [w1][w2][d2][d2] (host), theta [Dyl][d1][d2][Dyr], y [Dxl][d1][d2][Dxr].
 * y may not alias theta.  prec as in ite_debug_gemm. */
int ite_debug_heff_apply(ite_ctx* ctx, int Dxl, int Dyl, int Dxr, int Dyr, int d1, int d2,
                         int w0, int w1, int w2, const double* L, const double* W1h,
                         const double* W2h, const double* R, const double* theta,
                         double alpha, double beta, double* y, int prec);

/* The product of ite_debug_heff_apply as a local solve runs it (the MPO pair
 * matrix uploaded and, for prec 1 / 2, the environments rounded once, before
 * the timed region), repeated reps times on the context's stream; writes y
 * and the mean device time per product in milliseconds (HIP events). */
int ite_debug_heff_time(ite_ctx* ctx, int Dxl, int Dyl, int Dxr, int Dyr, int d1, int d2,
                        int w0, int w1, int w2, const double* L, const double* W1h,
                        const double* W2h, const double* R, const double* theta,
                        double alpha, double beta, double* y, int prec, int reps,
                        double* ms_per_product);

/* Environment updates (device pointers; W host):
 * dir = 0 (left):  E'[b', v, b] = sum E[a', w, a] X[a', p, b'] W[w, v, p, s] Y[a, s, b]
 *   E [Dxa][wl][Dya], X [Dxa][d][Dxb], Y [Dya][d][Dyb] -> E' [Dxb][wr][Dyb]
 * dir = 1 (right): E'[b', w, b] = sum E[c', v, c] X[b', p, c'] W[w, v, p, s] Y[b, s, c]
 *   E [Dxa][wr][Dya], X [Dxb][d][Dxa], Y [Dyb][d][Dya] -> E' [Dxb][wl][Dyb]
 * W == NULL means the overlap environment (no MPO index, wl = wr = 1). */
int ite_debug_env_update(ite_ctx* ctx, int dir, int Dxa, int Dya, int Dxb, int Dyb, int d,
                         int wl, int wr, const double* E, const double* X, const double* Wh,
                         const double* Y, double* Eout);

/* Truncated SVD split of theta [Dl][d1][d2][Dr] seen as an (Dl d1) x (d2 Dr)
 * matrix, by one-sided Jacobi: dir = 0 gives A1 = U, A2 = S V^T; dir = 1 gives
 * A1 = U S, A2 = V^T.  A1 [Dl][d1][k], A2 [k][d2][Dr] (device, capacity
 * min(rows, cols, chi_max) columns).  sigma_out (host, nullable, capacity
 * min(rows, cols)) receives all singular values in descending order; *k_out
 * and *disc_out (host) the kept count and discarded-weight fraction. */
int ite_debug_svd_split(ite_ctx* ctx, int dir, int Dl, int d1, int d2, int Dr,
                        const double* theta, int chi_max, double cutoff, double tie_rel,
                        double* A1, double* A2, double* sigma_out, int* k_out, double* disc_out);

/* One local solve: GMRES on (alpha I + beta H_eff) x = b with x0 as the
 * initial guess (shapes as ite_debug_heff_apply with Dyl = Dxl, Dyr = Dxr).
 * precision, max_refine, tol_refine as in ite_step_opts (mixed precision:
 * FP64 residuals, FP32 / BF16 GMRES corrections).  Writes x, the matvec count
 * (all precisions) and the final relative residual estimate. */
int ite_debug_local_solve(ite_ctx* ctx, int Dl, int Dr, int d1, int d2, int w0, int w1, int w2,
                          const double* L, const double* W1h, const double* W2h, const double* R,
                          double alpha, double beta, const double* b, const double* x0,
                          int krylov_dim, int max_cycles, double tol, int precision,
                          int max_refine, double tol_refine, double* x, int* matvecs,
                          double* res_rel);

/* One MFMA instruction of the given kind on fixed inputs, every lane's
 * accumulator written to out (host, 256 doubles for kind 0): used to check the
 * lane layout assumed by the GEMM kernels.  kind 0: FP64 16x16x4. */
int ite_debug_mfma_probe(ite_ctx* ctx, int kind, double* out);

#ifdef __cplusplus
}
#endif

#endif /* ITE_H */
