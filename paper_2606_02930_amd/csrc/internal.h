// Internal declarations of the implicit imaginary-time evolution library:
// error handling, the context (allocator, stream, workspaces) and the kernel
// launchers shared by the sweep engine.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <cstring>
#include <stdexcept>
#include <string>
#include <vector>

#include "ite.h"

namespace ite {

struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define ITE_FAIL(code, msg) throw ::ite::Error((code), (msg))
#define ITE_REQUIRE(cond, msg) \
    do { if (!(cond)) throw ::ite::Error(ITE_EINVAL, (msg)); } while (0)
// "file:line" of a failed call (the file's base name)
inline std::string src_loc(const char* file, int line) {
    const char* b = std::strrchr(file, '/');
    return std::string(b ? b + 1 : file) + ":" + std::to_string(line);
}
#define HIP_CHECK(expr)                                                                 \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            throw ::ite::Error(ITE_EDEVICE, std::string(#expr) + " failed (" +         \
                                                ::ite::src_loc(__FILE__, __LINE__) +    \
                                                "): " + hipGetErrorString(e_));         \
    } while (0)

// ---------------------------------------------------------------------------
// Kernel launchers (all asynchronous on `stream`)
// ---------------------------------------------------------------------------

// Operand precision of a contraction.
enum class Prec { F64 = 0, F32 = 1, BF16 = 2 };

// D[b] = alpha op(A[b]) op(B[b]) + beta C[b], row-major, b < batch.
// op(A) is M x K (A stored K x M when tA), op(B) is K x N (B stored N x K when
// tB).  C may be null (then beta is ignored).  D may alias C (same layout).
struct Gemm {
    int M = 0, N = 0, K = 0;
    bool tA = false, tB = false;
    double alpha = 1.0, beta = 0.0;
    const void* A = nullptr; long lda = 0, sA = 0;
    const void* B = nullptr; long ldb = 0, sB = 0;
    const double* C = nullptr; long ldc = 0, sC = 0;
    double* D = nullptr; long ldd = 0, sD = 0;
    int batch = 1;
    float* Df = nullptr;        // FP32 / BF16 operand kernels: FP32 output here instead of D (C must be null)
};
// FP64 operands, FP64 MFMA.
void gemm_f64(const Gemm& g, hipStream_t s);
// Split-K for under-filled products: the number of K parts (1 = no
// split) when the 128 x 128 output tiles of M x N fill at most half of
// `slots` concurrent workgroups and K is long; the parts (K / parts each, a
// multiple of the K slice) run as one batched launch into `work`
// (parts M N doubles) and are summed in a fixed order with alpha, beta, C.
int splitk_parts(int M, int N, int K, int slots);
void gemm_f64_splitk(const Gemm& g, int parts, double* work, hipStream_t s);
// The same with FP32 operands (FP32 accumulation within a part, the parts
// summed in FP64); FP64 output only.
void gemm_f32_splitk(const Gemm& g, int parts, double* work, hipStream_t s);
// Grouped FP64 GEMM: many problems (batch 1 each) in one persistent launch
// of `grid` workgroups, with bs x bs output tiles (128 or 64; the same bits
// either way).  The descriptors live in device memory (grouped_desc_bytes()
// each, filled on the host by grouped_desc_fill with the running tile count
// as tile_start); count (device) = {number of problems, their total tiles},
// so the same launch, e.g. inside a captured graph, serves changing problems.
size_t grouped_desc_bytes();
void grouped_desc_fill(const Gemm& g, int bs, int tile_start, void* out);
int grouped_tiles(const Gemm& g, int bs);
void gemm_grouped_f64(const void* desc, const int* count, bool tA, bool tB, int bs, int grid, hipStream_t s);
// The same for FP32 operands (FP32 MFMA, FP32 accumulation; output FP32 into
// Df or FP64 into D with alpha, beta, C), 128 x 128 tiles, A not transposed.
void gemm_grouped_f32(const void* desc, const int* count, bool tA, bool tB, int grid, hipStream_t s);
// FP32 operands (A, B are float*), FP32 MFMA, FP32 accumulation, FP64 output.
void gemm_f32(const Gemm& g, hipStream_t s);
// BF16 operands (A, B are uint16 bf16 bit patterns), BF16 MFMA, FP32
// accumulation, FP64 output.
void gemm_bf16(const Gemm& g, hipStream_t s);

// Small-matrix stage: out[g][o][c] = sum_i M[o][i] in[g][i][c] for a sparse
// M in CSR form.  Element addresses are two-level so that index permutations
// come for free:
//   in  + g*in_gs  + (i / in_div)*in_s1   + (i % in_div)*in_s2   + c*in_cs
//   out + g*out_gs + (o / out_div)*out_s1 + (o % out_div)*out_s2 + c*out_cs
struct Stage {
    int G = 0, I = 0, O = 0, C = 0;
    const double* in = nullptr;
    const float* in_f32 = nullptr;   // when set: FP32 input (same addressing) instead of `in`
    long in_gs = 0, in_s1 = 0, in_s2 = 0, in_cs = 1; int in_div = 1;
    double* out = nullptr;
    long out_gs = 0, out_s1 = 0, out_s2 = 0, out_cs = 1; int out_div = 1;
    const int* rowptr = nullptr; const int* col = nullptr; const double* val = nullptr;
    int nnz = -1;               // entries of the CSR matrix (-1: unknown, no LDS copy)
    int csr_lds = 0;            // set by the launcher: the matrix is copied to LDS
    int out_prec = 0;           // 0: FP64 into out; 1: FP32, 2: BF16 into out_lo
    void* out_lo = nullptr;
};
void stage_f64(const Stage& st, hipStream_t s);

// Rounding copies: FP64 -> FP32 and FP64 -> BF16 (round to nearest even).
void convert_f32(const double* x, float* y, size_t n, hipStream_t s);
void convert_bf16(const double* x, uint16_t* y, size_t n, hipStream_t s);

// Vector kernels.  Reductions are two-pass with a fixed grid so results do not
// depend on timing (bitwise reproducible for a given n).
int  reduce_blocks(size_t n);
// partial[b] = sum over block b of x.y
void dot_partials(const double* x, const double* y, size_t n, double* partial, hipStream_t s);
// partial[j*nb + b] = block b of V_j . w for j < k (V_j = V + j*ldv)
void mdot_partials(const double* V, long ldv, int k, const double* w, size_t n, double* partial,
                   hipStream_t s);
// out[j] (+)= sum_b partial[j*nb + b]; mode 0: store, 1: add, 2: store sqrt
void finish_partials(const double* partial, int k, int nb, double* out, int mode, hipStream_t s);
// w -= sum_j coef[j] V_j   (coef on device)
void gemv_sub(const double* V, long ldv, int k, const double* coef, double* w, size_t n,
              hipStream_t s);
// x += sum_j coef[j] V_j   (coef on device)
void gemv_add(const double* V, long ldv, int k, const double* coef, double* x, size_t n,
              hipStream_t s);
// out = a x + b y (host scalars; y may be null when b == 0)
void axpby(size_t n, double a, const double* x, double b, const double* y, double* out,
           hipStream_t s);
// out = x / *den (device scalar); writes zeros when *den <= thresh
void scale_inv(const double* x, const double* den, double* out, size_t n, hipStream_t s);
// One site of product-basis sampling (see sample_site_kernel): T [nsamples][d][Dr],
// u [nsamples], vnext [nsamples][Dr], cfg [nsamples][L]; d <= SAMPLE_DMAX.
constexpr int SAMPLE_DMAX = 16;
// flag (device, 2 values): flag[0] set to 1 when a sample's total probability
// is zero or not finite, flag[1] when its uniform is outside [0, 1).
void sample_site(const double* T, int nsamples, int d, int Dr, const double* u, double* vnext, int* cfg, int L,
                 int site, double* flag, hipStream_t s);
// Both classical Gram-Schmidt passes of one Arnoldi step in a single
// workgroup for n <= 8192 (k1 <= 64 basis vectors): coefficients to
// col[0..k1) and col[64..64+k1), ||w|| to col[128], vnext = w / ||w|| when
// not null.  Returns false (and does nothing) for longer vectors.
bool cgs2_small(const double* V, long ldv, int k1, double* w, size_t n, double* col, double* vnext, hipStream_t s);
// Device least-squares solve of one GMRES cycle (see hess_solve_one in
// vec.hip): hd holds the cycle's Hessenberg columns, HESS_HC doubles each,
// then ||b|| and ||r0||; y gets the mm combination coefficients; stats (8
// doubles per local solve, zeroed before the first cycle) accumulate the
// residual estimate, the product count and the flags.
constexpr int HESS_HC = 192, HESS_KMAX = 64;
void hess_solve(const double* hd, int mm, double* y, double* stats, bool r_product, bool last_cycle, hipStream_t s);
// Device eigensolve of a Lanczos cycle's projected matrix (lanczos_eig_kernel
// in vec.hip): y = the eigenvector of the lowest eigenvalue; rec: [0] the
// eigenvalue, [1] relative residual estimate, [2] += steps used, [3] steps used.
void lanczos_eig(const double* hd, int mm, double* y, double* rec, hipStream_t s);
// x *= a
void scale(double* x, double a, size_t n, hipStream_t s);
// y[i] = x[i*inc] for i < n (strided gather)
void fill(double* x, double v, size_t n, hipStream_t s);
// identity matrix D x D (row-major) into x
void eye(double* x, int D, hipStream_t s);
// sets *flag = 1 if any entry of x is not finite
void nonfinite_any(const double* x, size_t n, int* flag, hipStream_t s);
// out[j][i] = in[i][j]  (rows x cols -> cols x rows)
void transpose(const double* in, int rows, int cols, double* out, hipStream_t s);

// ---------------------------------------------------------------------------
// Batched fixed-budget GMRES: the local solves of several independent states
// advanced together, one launch per operation for all of them (persistent
// kernels over a fixed grid, problems described in device memory, so the
// same launches can be captured in a graph and replayed for other shapes).
// Per problem the arithmetic is that of the single-problem kernels above
// (the same reduction blocks and order), so a state's result does not depend
// on the batch it runs in.
// ---------------------------------------------------------------------------
struct BatchVec {
    long n;                 // vector length
    int nb;                 // reduction blocks, reduce_blocks(n)
    int small;              // Gram-Schmidt in one workgroup (cgs2_small applies)
    double* V;              // Krylov basis, (mm + 1) vectors of n
    double* w;              // work vector
    double* x;              // solution (in: initial guess)
    const double* b;        // right-hand side
    double* part;           // reduction partials, nb * 64 + 64
    double* hd;             // Hessenberg columns (mm x HESS_HC), ||b||, ||r0||
    double* y;              // combination coefficients (mm)
    double* stats;          // the solve's record (hess_solve)
    Stage st;               // MPO stage of the operator (X1 -> X3)
    // FP32 products (the refinement corrections of mixed precision): the
    // vector the product is applied to, rounded (n floats), and the stage
    // from FP32 X1 to FP32 X3
    float* tlo;
    Stage st_lo;
    int red_start, ew_start, stage_start;   // first unit of this problem in each unit range
};
// Unit totals of a batch (device ints): reductions, elementwise, stage.
enum { BT_RED = 0, BT_EW = 1, BT_STAGE = 2, BT_N = 4 };
constexpr int BATCH_GRID = 1024;      // workgroups of every batched vector launch
constexpr int BGRAPH_CACHE = 4;       // captured batched solves kept per context
constexpr long BATCH_EW = 4096;       // elements per elementwise unit
// Reductions: mode 0 V_j . w (j < k1; large problems), 1 w . w (large),
// 2 V_0 . V_0, 3 b . b (all problems).
void batch_reduce(const BatchVec* d, int G, const int* tot, int mode, int k1, hipStream_t s);
// Sum the partials: target 0 hd col k [j], 1 col k [64 + j], 2 col k [128]
// (sqrt; large problems), 3 ||b|| (sqrt), 4 ||r0|| (sqrt) (all).
void batch_finish(const BatchVec* d, int G, int k, int k1, int target, hipStream_t s);
// Elementwise: 0 w -= sum_(j <= k) col_k[j] V_j, 1 the same with col_k[64 + j]
// (large problems), 2 V_(k+1) = w / col_k[128] (large), 3 V_0 = b - V_0,
// 4 V_0 /= ||r0||, 5 x += sum_(j < k) y_j V_j, 6 tlo = V_k rounded to FP32
// (all).
void batch_vec(const BatchVec* d, int G, const int* tot, int op, int k, hipStream_t s);
// Both Gram-Schmidt passes of Arnoldi step k of the small problems.
void batch_cgs2_small(const BatchVec* d, int G, int k, int mm, hipStream_t s);
// The cycle's least-squares solve of every problem.
void batch_hess(const BatchVec* d, int G, int mm, bool r_product, bool last_cycle, hipStream_t s);
// Zero every problem's solve record (8 doubles).
void batch_zero_stats(const BatchVec* d, int G, hipStream_t s);
// The MPO stage of every problem (inputs per column at most 128).
void batch_stage(const BatchVec* d, int G, const int* tot, hipStream_t s);
// The FP32 stage st_lo of every problem (FP32 in, FP32 out).
void batch_stage_lo(const BatchVec* d, int G, const int* tot, hipStream_t s);
constexpr int BATCH_STAGE_SC = 128;

// Observability of kernel launches: every launch of a kind is counted, some
// are bracketed by events (begin returns true for those), and the
// algorithmic work actually done is added once it is known.
enum ProbeKind { PK_GEMM = 0, PK_GRAM = 1, PK_INNER = 2, PK_ROTATE = 3, PK_COUNT = 4 };
struct LaunchProbe {
    virtual ~LaunchProbe() = default;
    virtual bool begin(int kind, hipStream_t s) = 0;
    virtual void end(int kind, hipStream_t s) = 0;
    virtual void work(int kind, double flops, double bytes) = 0;
};

// One-sided Jacobi on the rows of Z[p][ld] (the first q columns are the
// matrix whose rows are orthogonalised; all ld columns are rotated).  probe
// may be null.
struct JacobiResult { int sweeps = 0; double last_off = 0.0; };
JacobiResult jacobi_rows(double* Z, int p, int q, int ld, double tol, int max_sweeps,
                         double* gram_ws, double* rot_ws, double* off_ws, double* host_off,
                         hipStream_t s, LaunchProbe* probe = nullptr);
// Build the Jacobi work matrix [theta | I_m] (dir 0) or [theta^T | I_n]
// (dir 1) for theta m x n; leading dimension m + n.
void jacobi_input(const double* theta, int m, int n, int dir, double* Z, hipStream_t s);
// Workspace sizes (doubles) of jacobi_rows for p rows of length q.
void jacobi_workspace(int p, int q, size_t* gram, size_t* rot, size_t* off);
// norms[i] = || Z[i][0:q] ||
void row_norms(const double* Z, int p, int q, int ld, double* norms, hipStream_t s);
// Gather kept rows: for t < k, r = perm[t]:
//   rowdst[t][0:nr] = Z[r][roff : roff + nr]
//   coldst[i][t]    = Z[r][coff + i] for i < nc   (a transposed write, ldc = k)
void gather_split(const double* Z, int ld, const int* perm, int k, int roff, int nr,
                  double* rowdst, int coff, int nc, double* coldst, hipStream_t s);

// Householder QR preconditioning of the Jacobi work matrix: Z <- Q^T Z with
// X = Q R the QR of the first q columns (p rows, leading dimension ld); the
// rows q..p-1 of the first part become zero when p > q.  Applies to
// 256 <= p <= 2048 and q >= 16; ws holds householder_workspace doubles.
bool householder_applies(int p, int q);
size_t householder_workspace(int p, int q, int ld);
void householder_rows(double* Z, int p, int q, int ld, double* ws, hipStream_t s);

// MFMA lane-layout probe (tests only).
void mfma_probe_f64(double* out, hipStream_t s);

}  // namespace ite
