// Bandwidth-bound kernels of the local solver: the Krylov vector operations
// of GMRES (dots, norms, classical Gram-Schmidt updates, combinations), the
// sparse MPO contraction stage, precision conversions and small helpers.
//
// Reductions are deterministic: a fixed number of blocks (a function of n
// only), a fixed per-block order (wavefront shuffles, then LDS), and a second
// pass that sums the block partials in index order.
#include "internal.h"
#include "wave.h"

#include <cmath>
#include <stdexcept>

namespace ite {
namespace {

constexpr int RT = 256;           // threads per reduction block
constexpr int MAX_RED_BLOCKS = 1024;

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Block sum of v (every thread of the block gets the result).
__device__ inline double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    const int nw = blockDim.x >> 6;
    for (int i = 0; i < nw; ++i) r += sh[i];
    return r;
}

// Block vb of a reduction over vg blocks (the partition depends on n only,
// through vg = reduce_blocks(n)): *out = the block's share of x . y.
__device__ inline void dot_block(const double* __restrict__ x, const double* __restrict__ y, size_t n, int vb, int vg,
                                 double* __restrict__ out, double* sh) {
    double acc = 0.0;
    const size_t stride = (size_t)vg * RT;
    for (size_t i = (size_t)vb * RT + threadIdx.x; i < n; i += stride) acc += x[i] * y[i];
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) *out = acc;
}

__global__ __launch_bounds__(RT) void dot_partials_kernel(const double* __restrict__ x,
                                                          const double* __restrict__ y, size_t n,
                                                          double* __restrict__ partial) {
    __shared__ double sh[RT / 64];
    dot_block(x, y, n, blockIdx.x, gridDim.x, partial + blockIdx.x, sh);
}

// Block vb of vg: partial[j * vg + vb] = its share of V_j . w for j < k.
template <int KMAX>
__device__ inline void mdot_block(const double* __restrict__ V, long ldv, int k, const double* __restrict__ w, size_t n,
                                  int vb, int vg, double* __restrict__ partial, double* sh) {
    double acc[KMAX];
#pragma unroll
    for (int j = 0; j < KMAX; ++j) acc[j] = 0.0;
    const size_t stride = (size_t)vg * RT;
    for (size_t i = (size_t)vb * RT + threadIdx.x; i < n; i += stride) {
        const double wi = w[i];
#pragma unroll
        for (int j = 0; j < KMAX; ++j)
            if (j < k) acc[j] += V[(size_t)j * ldv + i] * wi;
    }
    for (int j = 0; j < k; ++j) {
        const double s = block_sum(acc[j], sh);
        if (threadIdx.x == 0) partial[(size_t)j * vg + vb] = s;
    }
}

// partial[j*nb + b]: block b's share of V_j . w for j < k (k <= 64).
template <int KMAX>
__global__ __launch_bounds__(RT) void mdot_partials_kernel(const double* __restrict__ V, long ldv,
                                                           int k, const double* __restrict__ w,
                                                           size_t n, double* __restrict__ partial) {
    __shared__ double sh[RT / 64];
    mdot_block<KMAX>(V, ldv, k, w, n, blockIdx.x, gridDim.x, partial, sh);
}

// *out (mode 0: =, 1: +=, 2: = sqrt) of the sum of nb partials.
__device__ inline void finish_one(const double* __restrict__ partial, int nb, double* __restrict__ out, int mode,
                                  double* sh) {
    double acc = 0.0;
    // fixed assignment of partials to threads, fixed combination order
    for (int b = threadIdx.x; b < nb; b += RT) acc += partial[b];
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) {
        if (mode == 0) *out = acc;
        else if (mode == 1) *out += acc;
        else *out = sqrt(fmax(acc, 0.0));
    }
}

__global__ __launch_bounds__(RT) void finish_partials_kernel(const double* __restrict__ partial,
                                                             int nb, double* __restrict__ out,
                                                             int mode) {
    __shared__ double sh[RT / 64];
    const int j = blockIdx.x;
    finish_one(partial + (size_t)j * nb, nb, out + j, mode, sh);
}

template <int KMAX, bool SUB>
__global__ __launch_bounds__(RT) void gemv_kernel(const double* __restrict__ V, long ldv, int k,
                                                  const double* __restrict__ coef,
                                                  double* __restrict__ w, size_t n) {
    double c[KMAX];
#pragma unroll
    for (int j = 0; j < KMAX; ++j) c[j] = (j < k) ? coef[j] : 0.0;
    const size_t stride = (size_t)gridDim.x * RT;
    for (size_t i = (size_t)blockIdx.x * RT + threadIdx.x; i < n; i += stride) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < KMAX; ++j)
            if (j < k) s += c[j] * V[(size_t)j * ldv + i];
        w[i] = SUB ? w[i] - s : w[i] + s;
    }
}

__global__ void axpby_kernel(size_t n, double a, const double* __restrict__ x, double b,
                             const double* __restrict__ y, double* __restrict__ out) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        out[i] = y ? a * x[i] + b * y[i] : a * x[i];
}

// Both Gram-Schmidt passes of one Arnoldi step for short vectors, in one
// workgroup: w <- w - V (V^T w) twice (V: k1 vectors of length n, leading
// dimension ldv), the coefficients of the passes to col[0..k1) and
// col[64..64+k1), ||w|| to col[128] and, when vnext is given,
// vnext = w / ||w|| (0 for a zero norm, as scale_inv).  Thread t owns the
// entries t, t + CGS_T, ... of w, kept in LDS between the passes; fixed
// reduction order.
constexpr int CGS_T = 256, CGS_E = 32;
template <int KMAX>
struct CgsLDS {
    double xs[CGS_T * CGS_E];
    double part[CGS_T / 64][KMAX];
    double coef[KMAX];
};
template <int KMAX>
__device__ inline void cgs2_small_body(const double* __restrict__ V, long ldv, int k1, double* __restrict__ w, int n,
                                       double* __restrict__ col, double* __restrict__ vnext, CgsLDS<KMAX>& L) {
    auto& xs = L.xs;
    auto& part = L.part;
    auto& coef = L.coef;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    for (int i = t; i < n; i += CGS_T) xs[i] = w[i];
    for (int pass = 0; pass < 2; ++pass) {
        double acc[KMAX];
#pragma unroll
        for (int j = 0; j < KMAX; ++j) acc[j] = 0.0;
        for (int i = t; i < n; i += CGS_T) {
            const double xi = xs[i];
#pragma unroll
            for (int j = 0; j < KMAX; ++j)
                if (j < k1) acc[j] += V[j * ldv + i] * xi;
        }
#pragma unroll
        for (int j = 0; j < KMAX; ++j) {
            if (j < k1) {
                const double sj = wave_sum(acc[j]);
                if (lane == 0) part[wv][j] = sj;
            }
        }
        __syncthreads();
        if (t < k1) {
            double sj = 0.0;
#pragma unroll
            for (int ww = 0; ww < CGS_T / 64; ++ww) sj += part[ww][t];
            coef[t] = sj;
            col[64 * pass + t] = sj;
        }
        __syncthreads();
        for (int i = t; i < n; i += CGS_T) {
            double xi = xs[i];
#pragma unroll
            for (int j = 0; j < KMAX; ++j)
                if (j < k1) xi -= coef[j] * V[j * ldv + i];
            xs[i] = xi;
        }
        __syncthreads();
    }
    double ss = 0.0;
    for (int i = t; i < n; i += CGS_T) ss += xs[i] * xs[i];
    ss = wave_sum(ss);
    if (lane == 0) part[wv][0] = ss;
    __syncthreads();
    double tot = 0.0;
#pragma unroll
    for (int ww = 0; ww < CGS_T / 64; ++ww) tot += part[ww][0];
    const double nrm = sqrt(fmax(tot, 0.0));
    if (t == 0) col[128] = nrm;
    const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
    for (int i = t; i < n; i += CGS_T) {
        w[i] = xs[i];
        if (vnext) vnext[i] = xs[i] * inv;
    }
}

template <int KMAX>
__global__ __launch_bounds__(CGS_T) void cgs2_small_kernel(const double* __restrict__ V, long ldv, int k1,
                                                           double* __restrict__ w, int n, double* __restrict__ col,
                                                           double* __restrict__ vnext) {
    __shared__ CgsLDS<KMAX> sh;
    cgs2_small_body<KMAX>(V, ldv, k1, w, n, col, vnext, sh);
}

// The small least-squares problem of one GMRES cycle, on the device (one
// thread; the Hessenberg matrix in LDS): the columns of the cycle's Arnoldi
// steps are hd[k * HESS_HC + i] (first Gram-Schmidt pass), + 64 (second
// pass), + 128 (the norm of the next vector); hd[mm * HESS_HC] = ||b||,
// hd[mm * HESS_HC + 1] = beta = ||r0||.  Givens rotations reduce H to upper
// triangular form while the residual estimate |g_(k+1)| is tracked; an
// Arnoldi step whose next norm is <= 1e-14 beta ends the cycle (invariant
// subspace); y solves R y = g by back substitution (zero beyond the steps
// used).  stats (per local solve, zeroed by the caller before the first
// cycle): [0] relative residual estimate, [1] products whose results enter
// the solution, [2] ITE_FLAG_* bits, [3] 1 once a cycle found an invariant
// subspace or a zero residual (later cycles then change nothing).
// LDS of one solve: H ((KMAX + 1) x KMAX), then cos, sin and g.
constexpr int HESS_LDS = (HESS_KMAX + 1) * HESS_KMAX + 3 * HESS_KMAX + 1;
__device__ void hess_solve_one(const double* __restrict__ hd, int mm, double* __restrict__ y,
                               double* __restrict__ stats, int r_product, int last_cycle, double* Hs) {
    if (stats[3] != 0.0) {
        for (int i = 0; i < mm; ++i) y[i] = 0.0;
        return;
    }
    if (r_product) {
        stats[1] += 1.0;
        stats[4] += 1.0;   // the residual products alone (FP64 even when the others are not)
    }
    const double bnorm = hd[(size_t)mm * HESS_HC], beta = hd[(size_t)mm * HESS_HC + 1];
    stats[0] = bnorm > 0.0 ? beta / bnorm : 0.0;
    if (!(beta > 0.0)) {
        for (int i = 0; i < mm; ++i) y[i] = 0.0;
        stats[3] = 1.0;
        return;
    }
    double* cs = Hs + (HESS_KMAX + 1) * HESS_KMAX;
    double* sn = cs + HESS_KMAX;
    double* g = sn + HESS_KMAX;
    for (int i = 0; i <= mm; ++i) g[i] = 0.0;
    g[0] = beta;
    int kused = 0;
    bool breakdown = false;
    for (int k = 0; k < mm; ++k) {
        const double* col = hd + (size_t)k * HESS_HC;
        for (int i = 0; i <= k; ++i) Hs[i * HESS_KMAX + k] = col[i] + col[64 + i];
        const double hnext = col[128];
        for (int i = 0; i < k; ++i) {
            const double a = Hs[i * HESS_KMAX + k], bb = Hs[(i + 1) * HESS_KMAX + k];
            Hs[i * HESS_KMAX + k] = cs[i] * a + sn[i] * bb;
            Hs[(i + 1) * HESS_KMAX + k] = -sn[i] * a + cs[i] * bb;
        }
        const double a = Hs[k * HESS_KMAX + k];
        const double rr = hypot(a, hnext);
        cs[k] = rr > 0.0 ? a / rr : 1.0;
        sn[k] = rr > 0.0 ? hnext / rr : 0.0;
        Hs[k * HESS_KMAX + k] = rr;
        g[k + 1] = -sn[k] * g[k];
        g[k] = cs[k] * g[k];
        kused = k + 1;
        stats[0] = bnorm > 0.0 ? fabs(g[k + 1]) / bnorm : 0.0;
        if (hnext <= 1e-14 * beta) {
            breakdown = true;
            break;
        }
    }
    stats[1] += kused;
    for (int i = kused - 1; i >= 0; --i) {
        double sum = g[i];
        for (int j = i + 1; j < kused; ++j) sum -= Hs[i * HESS_KMAX + j] * y[j];
        const double dgn = Hs[i * HESS_KMAX + i];
        y[i] = dgn != 0.0 ? sum / dgn : 0.0;
    }
    for (int i = kused; i < mm; ++i) y[i] = 0.0;
    int flags = (int)stats[2];
    if (breakdown) {
        flags |= ITE_FLAG_BREAKDOWN;
        stats[3] = 1.0;
    } else if (last_cycle) {
        flags |= ITE_FLAG_BUDGET_EXHAUSTED;
    }
    stats[2] = (double)flags;
}

__global__ __launch_bounds__(64) void hess_solve_kernel(const double* __restrict__ hd, int mm, double* __restrict__ y,
                                                        double* __restrict__ stats, int r_product, int last_cycle) {
    __shared__ double Hs[HESS_LDS];
    if (threadIdx.x == 0) hess_solve_one(hd, mm, y, stats, r_product, last_cycle, Hs);
}

__global__ void scale_inv_kernel(const double* __restrict__ x, const double* __restrict__ den,
                                 double* __restrict__ out, size_t n) {
    const double d = *den;
    const double inv = d > 0.0 ? 1.0 / d : 0.0;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        out[i] = x[i] * inv;
}

__global__ void scale_kernel(double* __restrict__ x, double a, size_t n) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) x[i] *= a;
}

__global__ void fill_kernel(double* __restrict__ x, double v, size_t n) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) x[i] = v;
}

__global__ void eye_kernel(double* __restrict__ x, int D) {
    const size_t n = (size_t)D * D;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        x[i] = (i / D == i % D) ? 1.0 : 0.0;
}

__global__ void nonfinite_kernel(const double* __restrict__ x, size_t n, int* flag) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    bool bad = false;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        bad |= !isfinite(x[i]);
    if (bad) atomicOr(flag, 1);
}

__global__ void f32_kernel(const double* __restrict__ x, float* __restrict__ y, size_t n) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        y[i] = (float)x[i];
}

// FP64 -> BF16 with round to nearest even, done in two exact steps: the FP64
// value is first rounded to FP32 with round-to-odd (so that the second
// rounding cannot double-round), then FP32 -> BF16 by the usual
// add-0x7fff-plus-lsb rule.  NaN stays NaN.
__device__ inline uint16_t to_bf16(double v) {
    float f = (float)v;
    if (isfinite(f) && (double)f != v) {
        // round to odd: truncate toward zero, then set the last bit
        uint32_t u = __float_as_uint(f);
        if (fabs((double)f) > fabs(v)) u -= 1;   // move toward zero
        u |= 1u;
        f = __uint_as_float(u);
    }
    uint32_t u = __float_as_uint(f);
    if (isnan(f)) return (uint16_t)((u >> 16) | 0x40);
    const uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (uint16_t)(u >> 16);
}

__global__ void bf16_kernel(const double* __restrict__ x, uint16_t* __restrict__ y, size_t n) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        y[i] = to_bf16(x[i]);
}

// out[j][i] = in[i][j] through a 32 x 32 LDS tile.
__global__ void transpose_kernel(const double* __restrict__ in, int rows, int cols,
                                 double* __restrict__ out) {
    __shared__ double tile[32][33];
    const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
    for (int k = threadIdx.y; k < 32; k += blockDim.y) {
        const int r = r0 + k, c = c0 + threadIdx.x;
        if (r < rows && c < cols) tile[k][threadIdx.x] = in[(size_t)r * cols + c];
    }
    __syncthreads();
    for (int k = threadIdx.y; k < 32; k += blockDim.y) {
        const int c = c0 + k, r = r0 + threadIdx.x;
        if (r < rows && c < cols) out[(size_t)c * rows + r] = tile[threadIdx.x][k];
    }
}

// ---------------------------------------------------------------------------
// Sparse MPO stage.  A block handles one g and SC consecutive columns; the
// I inputs of those columns are staged in LDS, then every thread produces the
// O outputs of its column from the CSR rows (uniform across the block, so the
// matrix entries come through scalar loads).  SC shrinks with I so that the
// staged inputs stay within 128 KiB of LDS: SC = 128 up to 128 inputs, down
// to 16 columns for the largest stage an MPO can have (w = 16, d = 8: 1024).
// ---------------------------------------------------------------------------
constexpr size_t STAGE_LDS = 128 * 1024;
// LDS of a stage workgroup: the inputs (at most STAGE_LDS) and, when it fits,
// the CSR matrix behind them
constexpr size_t STAGE_LDS_TOTAL = 152 * 1024;

// OUT: 0 writes FP64 to st.out, 1 rounds to FP32 and 2 to BF16 into st.out_lo
// (the operand of a following low-precision contraction).
template <int OUT, int SC>
__device__ inline void stage_unit(const Stage& st, int g, int cblk, double* xin) {
    const int c = cblk * SC + threadIdx.x;
    const long cin = (long)g * st.in_gs + (long)c * st.in_cs;
    if (st.in_f32) {
        const float* __restrict__ in = st.in_f32 + cin;
        for (int i = 0; i < st.I; ++i) {
            const long off = (long)(i / st.in_div) * st.in_s1 + (long)(i % st.in_div) * st.in_s2;
            xin[i * SC + threadIdx.x] = (c < st.C) ? (double)in[off] : 0.0;
        }
    } else {
        const double* __restrict__ in = st.in + cin;
        for (int i = 0; i < st.I; ++i) {
            const long off = (long)(i / st.in_div) * st.in_s1 + (long)(i % st.in_div) * st.in_s2;
            xin[i * SC + threadIdx.x] = (c < st.C) ? in[off] : 0.0;
        }
    }
    // the CSR matrix in LDS when it fits behind the inputs (read as
    // broadcasts instead of a chain of dependent scalar loads)
    const int nnz = st.nnz;
    const bool lcsr = st.csr_lds != 0;
    double* sval = xin + (size_t)st.I * SC;
    int* scol = reinterpret_cast<int*>(sval + nnz);
    int* srow = scol + nnz;
    if (lcsr) {
        for (int e = threadIdx.x; e < nnz; e += SC) {
            sval[e] = st.val[e];
            scol[e] = st.col[e];
        }
        for (int o = threadIdx.x; o <= st.O; o += SC) srow[o] = st.rowptr[o];
    }
    __syncthreads();
    if (c < st.C) {
        const long base = (long)g * st.out_gs + (long)c * st.out_cs;
        const int* rp = lcsr ? srow : st.rowptr;
        const int* cl = lcsr ? scol : st.col;
        const double* vl = lcsr ? sval : st.val;
        for (int o = 0; o < st.O; ++o) {
            double acc = 0.0;
            const int e1 = rp[o + 1];
            for (int e = rp[o]; e < e1; ++e) acc += vl[e] * xin[cl[e] * SC + threadIdx.x];
            const long at = base + (long)(o / st.out_div) * st.out_s1 + (long)(o % st.out_div) * st.out_s2;
            if (OUT == 0) st.out[at] = acc;
            else if (OUT == 1) static_cast<float*>(st.out_lo)[at] = (float)acc;
            else static_cast<uint16_t*>(st.out_lo)[at] = to_bf16(acc);
        }
    }
    __syncthreads();   // xin may be refilled by the caller's next unit
}

template <int OUT, int SC>
__global__ __launch_bounds__(SC) void stage_kernel(Stage st) {
    extern __shared__ double xin[];   // [I][SC]
    stage_unit<OUT, SC>(st, blockIdx.y, blockIdx.x, xin);
}

// Four adjacent columns per thread (unit column strides, every stride a
// multiple of 4, 16-byte aligned bases): 16-byte loads and stores instead of
// one element per lane.  The inputs keep their type in LDS (an FP32 input
// takes half the space, so twice the columns fit per compute unit), laid out
// [I][4][SC] so that each LDS read is lane-contiguous.  Same sums in the same
// order as stage_unit.
template <typename TIN>
__device__ inline void load4(const TIN* p, TIN (&v)[4]) {
    if constexpr (sizeof(TIN) == 4) {
        const float4 q = *reinterpret_cast<const float4*>(p);
        v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
    } else {
        const double2 a = *reinterpret_cast<const double2*>(p);
        const double2 b = *reinterpret_cast<const double2*>(p + 2);
        v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
    }
}

template <int OUT, int SC, typename TIN>
__global__ __launch_bounds__(SC) void stage4_kernel(Stage st) {
    extern __shared__ double lds_raw[];
    TIN* xin = reinterpret_cast<TIN*>(lds_raw);   // [I][4][SC]
    const int g = blockIdx.y;
    const int t = threadIdx.x;
    const int c0 = (blockIdx.x * SC + t) * 4;
    const bool live = c0 < st.C;
    const TIN* __restrict__ in;
    if constexpr (sizeof(TIN) == 4) in = st.in_f32;
    else in = st.in;
    in += (long)g * st.in_gs + c0;
    const bool in_flat = st.in_div == 1;   // no division in the common layout
    for (int i = 0; i < st.I; ++i) {
        TIN v[4] = {0, 0, 0, 0};
        const long off = in_flat ? (long)i * st.in_s1
                                 : (long)(i / st.in_div) * st.in_s1 + (long)(i % st.in_div) * st.in_s2;
        if (live) load4(in + off, v);
#pragma unroll
        for (int q = 0; q < 4; ++q) xin[(i * 4 + q) * SC + t] = v[q];
    }
    const int nnz = st.nnz;
    const bool lcsr = st.csr_lds != 0;
    double* sval = reinterpret_cast<double*>(xin + (size_t)st.I * 4 * SC);
    int* scol = reinterpret_cast<int*>(sval + nnz);
    int* srow = scol + nnz;
    if (lcsr) {
        for (int e = t; e < nnz; e += SC) {
            sval[e] = st.val[e];
            scol[e] = st.col[e];
        }
        for (int o = t; o <= st.O; o += SC) srow[o] = st.rowptr[o];
    }
    __syncthreads();
    if (!live) return;
    const int* rp = lcsr ? srow : st.rowptr;
    const int* cl = lcsr ? scol : st.col;
    const double* vl = lcsr ? sval : st.val;
    const long base = (long)g * st.out_gs + c0;
    const bool out_flat = st.out_div == 1;
    for (int o = 0; o < st.O; ++o) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        const int e1 = rp[o + 1];
        for (int e = rp[o]; e < e1; ++e) {
            const double w = vl[e];
            const TIN* x = xin + cl[e] * 4 * SC + t;
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] += w * (double)x[q * SC];
        }
        const long at = base + (out_flat ? (long)o * st.out_s1
                                         : (long)(o / st.out_div) * st.out_s1 + (long)(o % st.out_div) * st.out_s2);
        if (OUT == 0) {
            *reinterpret_cast<double2*>(st.out + at) = double2{acc[0], acc[1]};
            *reinterpret_cast<double2*>(st.out + at + 2) = double2{acc[2], acc[3]};
        } else if (OUT == 1) {
            *reinterpret_cast<float4*>(static_cast<float*>(st.out_lo) + at) =
                float4{(float)acc[0], (float)acc[1], (float)acc[2], (float)acc[3]};
        } else {
            uint2 v;
            v.x = (uint32_t)to_bf16(acc[0]) | ((uint32_t)to_bf16(acc[1]) << 16);
            v.y = (uint32_t)to_bf16(acc[2]) | ((uint32_t)to_bf16(acc[3]) << 16);
            *reinterpret_cast<uint2*>(static_cast<uint16_t*>(st.out_lo) + at) = v;
        }
    }
}

inline int grid_for(size_t n, int threads, int cap = 4096) {
    size_t b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > (size_t)cap) b = cap;
    return (int)b;
}

}  // namespace

int reduce_blocks(size_t n) {
    size_t b = (n + RT * 4 - 1) / (RT * 4);
    if (b < 1) b = 1;
    if (b > MAX_RED_BLOCKS) b = MAX_RED_BLOCKS;
    return (int)b;
}

void dot_partials(const double* x, const double* y, size_t n, double* partial, hipStream_t s) {
    hipLaunchKernelGGL(dot_partials_kernel, dim3(reduce_blocks(n)), dim3(RT), 0, s, x, y, n, partial);
    HIP_CHECK(hipGetLastError());
}

void mdot_partials(const double* V, long ldv, int k, const double* w, size_t n, double* partial,
                   hipStream_t s) {
    const int nb = reduce_blocks(n);
    if (k <= 4)
        hipLaunchKernelGGL((mdot_partials_kernel<4>), dim3(nb), dim3(RT), 0, s, V, ldv, k, w, n, partial);
    else if (k <= 8)
        hipLaunchKernelGGL((mdot_partials_kernel<8>), dim3(nb), dim3(RT), 0, s, V, ldv, k, w, n, partial);
    else if (k <= 16)
        hipLaunchKernelGGL((mdot_partials_kernel<16>), dim3(nb), dim3(RT), 0, s, V, ldv, k, w, n, partial);
    else {
        // wider bases: 16 at a time
        for (int j0 = 0; j0 < k; j0 += 16) {
            const int kk = k - j0 < 16 ? k - j0 : 16;
            hipLaunchKernelGGL((mdot_partials_kernel<16>), dim3(nb), dim3(RT), 0, s, V + (size_t)j0 * ldv,
                               ldv, kk, w, n, partial + (size_t)j0 * nb);
        }
    }
    HIP_CHECK(hipGetLastError());
}

void finish_partials(const double* partial, int k, int nb, double* out, int mode, hipStream_t s) {
    hipLaunchKernelGGL(finish_partials_kernel, dim3(k), dim3(RT), 0, s, partial, nb, out, mode);
    HIP_CHECK(hipGetLastError());
}

template <bool SUB>
static void gemv_launch(const double* V, long ldv, int k, const double* coef, double* w, size_t n,
                        hipStream_t s) {
    const int nb = grid_for(n, RT);
    for (int j0 = 0; j0 < k; j0 += 16) {
        const int kk = k - j0 < 16 ? k - j0 : 16;
        if (kk <= 4)
            hipLaunchKernelGGL((gemv_kernel<4, SUB>), dim3(nb), dim3(RT), 0, s, V + (size_t)j0 * ldv, ldv, kk,
                               coef + j0, w, n);
        else if (kk <= 8)
            hipLaunchKernelGGL((gemv_kernel<8, SUB>), dim3(nb), dim3(RT), 0, s, V + (size_t)j0 * ldv, ldv, kk,
                               coef + j0, w, n);
        else
            hipLaunchKernelGGL((gemv_kernel<16, SUB>), dim3(nb), dim3(RT), 0, s, V + (size_t)j0 * ldv, ldv, kk,
                               coef + j0, w, n);
    }
    HIP_CHECK(hipGetLastError());
}

void gemv_sub(const double* V, long ldv, int k, const double* coef, double* w, size_t n, hipStream_t s) {
    gemv_launch<true>(V, ldv, k, coef, w, n, s);
}
void gemv_add(const double* V, long ldv, int k, const double* coef, double* x, size_t n, hipStream_t s) {
    gemv_launch<false>(V, ldv, k, coef, x, n, s);
}

void axpby(size_t n, double a, const double* x, double b, const double* y, double* out, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(axpby_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, n, a, x, b, y, out);
    HIP_CHECK(hipGetLastError());
}

bool cgs2_small(const double* V, long ldv, int k1, double* w, size_t n, double* col, double* vnext, hipStream_t s) {
    if (n == 0 || n > (size_t)CGS_T * CGS_E || k1 < 1 || k1 > 64) return false;
    const int nn = (int)n;
    if (k1 <= 8)
        hipLaunchKernelGGL((cgs2_small_kernel<8>), dim3(1), dim3(CGS_T), 0, s, V, ldv, k1, w, nn, col, vnext);
    else if (k1 <= 16)
        hipLaunchKernelGGL((cgs2_small_kernel<16>), dim3(1), dim3(CGS_T), 0, s, V, ldv, k1, w, nn, col, vnext);
    else if (k1 <= 32)
        hipLaunchKernelGGL((cgs2_small_kernel<32>), dim3(1), dim3(CGS_T), 0, s, V, ldv, k1, w, nn, col, vnext);
    else
        hipLaunchKernelGGL((cgs2_small_kernel<64>), dim3(1), dim3(CGS_T), 0, s, V, ldv, k1, w, nn, col, vnext);
    HIP_CHECK(hipGetLastError());
    return true;
}

// One site of the conditional sampling of an MPS in the product basis, one
// workgroup per sample: T[smp] ([d][Dr]) = v A_site for that sample's
// normalised left vector v; p_s = ||T[smp][s]||^2 (fixed reduction order);
// the site takes the first s with p_0 + .. + p_s > u[smp] (p_0 + .. + p_(d-1))
// and p_s > 0 (else the last s with p_s > 0, else 0), written to
// cfg[smp * L + site]; vnext[smp] = T[smp][s] / ||T[smp][s]||.  A total that
// is zero or not finite (a zero or non-finite state) sets flag[0] = 1, a
// uniform outside [0, 1) flag[1] = 1.
constexpr int SMP_T = 256;
__global__ __launch_bounds__(SMP_T) void sample_site_kernel(const double* __restrict__ T, int d, int Dr,
                                                            const double* __restrict__ u,
                                                            double* __restrict__ vnext, int* __restrict__ cfg,
                                                            int L, int site, double* __restrict__ flag) {
    __shared__ double part[SMP_T / 64][SAMPLE_DMAX];
    __shared__ double pw[SAMPLE_DMAX];
    __shared__ int chosen;
    const int smp = blockIdx.x, t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const double* row = T + (size_t)smp * d * Dr;
    for (int q = 0; q < d; ++q) {
        double acc = 0.0;
        for (int j = t; j < Dr; j += SMP_T) {
            const double x = row[(size_t)q * Dr + j];
            acc += x * x;
        }
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);   // butterfly: fixed order
        if (lane == 0) part[wv][q] = acc;
    }
    __syncthreads();
    if (t == 0) {
        double tot = 0.0;
        for (int q = 0; q < d; ++q) {
            double pq = 0.0;
            for (int w = 0; w < SMP_T / 64; ++w) pq += part[w][q];
            pw[q] = pq;
            tot += pq;
        }
        if (!(tot > 0.0) || !isfinite(tot)) flag[0] = 1.0;
        if (!(u[smp] >= 0.0 && u[smp] < 1.0)) flag[1] = 1.0;
        const double thr = u[smp] * tot;
        int pick = -1;
        double cum = 0.0;
        for (int q = 0; q < d; ++q) {
            cum += pw[q];
            if (pick < 0 && cum > thr && pw[q] > 0.0) pick = q;
        }
        for (int q = d - 1; q >= 0 && pick < 0; --q)
            if (pw[q] > 0.0) pick = q;
        if (pick < 0) pick = 0;
        chosen = pick;
        cfg[(size_t)smp * L + site] = pick;
    }
    __syncthreads();
    const int q = chosen;
    const double nq = pw[q];
    const double inv = nq > 0.0 ? 1.0 / sqrt(nq) : 0.0;
    for (int j = t; j < Dr; j += SMP_T) vnext[(size_t)smp * Dr + j] = row[(size_t)q * Dr + j] * inv;
}

void sample_site(const double* T, int nsamples, int d, int Dr, const double* u, double* vnext, int* cfg, int L,
                 int site, double* flag, hipStream_t s) {
    if (nsamples <= 0) return;
    if (d < 1 || d > SAMPLE_DMAX || Dr < 1) throw std::invalid_argument("sample_site: bad dimensions");
    hipLaunchKernelGGL(sample_site_kernel, dim3(nsamples), dim3(SMP_T), 0, s, T, d, Dr, u, vnext, cfg, L, site,
                       flag);
    HIP_CHECK(hipGetLastError());
}

void scale_inv(const double* x, const double* den, double* out, size_t n, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(scale_inv_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, x, den, out, n);
    HIP_CHECK(hipGetLastError());
}

// Lowest eigenpair of the Lanczos cycle's projected matrix, on the device
// (one wavefront): T (kused x kused, symmetric) from the Gram-Schmidt
// coefficients of the columns hd[k * HESS_HC ..] (both passes summed, the
// upper triangle mirrored), kused the steps up to the first breakdown (a
// next norm <= 1e-14 of the largest diagonal so far); cyclic Jacobi rotations
// (each zeroes t_pq with tan the smaller root of t^2 + 2 tau t - 1 = 0,
// tau = (t_qq - t_pp) / (2 t_pq)) until the off-diagonal mass is below 1e-32
// of the total (at most 60 sweeps); y = the eigenvector of the smallest
// eigenvalue (zero beyond kused).  rec: [0] the eigenvalue, [1] the residual
// estimate |h_(k+1,k) y_k| / |theta| (its absolute value when theta = 0),
// [2] += kused, [3] kused.
__global__ __launch_bounds__(64) void lanczos_eig_kernel(const double* __restrict__ hd, int mm,
                                                         double* __restrict__ y, double* __restrict__ rec) {
    __shared__ double A[HESS_KMAX][HESS_KMAX + 1];
    __shared__ double Z[HESS_KMAX][HESS_KMAX + 1];
    __shared__ double cs[2];
    __shared__ int ku;
    __shared__ double red[2];
    const int t = threadIdx.x;
    if (t == 0) {
        int kused = mm;
        double scale_h = 0.0;
        for (int k = 0; k < mm; ++k) {
            const double* col = hd + (size_t)k * HESS_HC;
            scale_h = fmax(scale_h, fabs(col[k] + col[64 + k]));
            if (k + 1 < mm && !(col[128] > 1e-14 * fmax(scale_h, 1e-300))) {
                kused = k + 1;
                break;
            }
        }
        ku = kused;
    }
    __syncthreads();
    const int k = ku;
    for (int c = 0; c < k; ++c) {
        const double* col = hd + (size_t)c * HESS_HC;
        if (t <= c) {
            const double v = col[t] + col[64 + t];
            A[t][c] = v;
            A[c][t] = v;
        }
        if (t < k) Z[c][t] = c == t ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int sweep = 0; sweep < 60; ++sweep) {
        if (t == 0) {
            double off = 0.0, tot = 0.0;
            for (int i = 0; i < k; ++i)
                for (int j = 0; j < k; ++j) {
                    const double v = A[i][j] * A[i][j];
                    tot += v;
                    if (i != j) off += v;
                }
            red[0] = off;
            red[1] = tot;
        }
        __syncthreads();
        if (!(red[0] > 1e-32 * red[1])) break;
        for (int p = 0; p < k; ++p)
            for (int q = p + 1; q < k; ++q) {
                if (t == 0) {
                    const double apq = A[p][q];
                    double cc = 1.0, ss = 0.0;
                    if (apq != 0.0) {
                        const double tau = (A[q][q] - A[p][p]) / (2.0 * apq);
                        const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        cc = 1.0 / sqrt(1.0 + tt * tt);
                        ss = tt * cc;
                    }
                    cs[0] = cc;
                    cs[1] = ss;
                }
                __syncthreads();
                const double cc = cs[0], ss = cs[1];
                if (ss != 0.0) {
                    if (t < k) {   // columns p, q of A J
                        const double arp = A[t][p], arq = A[t][q];
                        A[t][p] = cc * arp - ss * arq;
                        A[t][q] = ss * arp + cc * arq;
                    }
                    __syncthreads();
                    if (t < k) {   // rows p, q of J^T (A J); Z J
                        const double apr = A[p][t], aqr = A[q][t];
                        A[p][t] = cc * apr - ss * aqr;
                        A[q][t] = ss * apr + cc * aqr;
                        const double zrp = Z[t][p], zrq = Z[t][q];
                        Z[t][p] = cc * zrp - ss * zrq;
                        Z[t][q] = ss * zrp + cc * zrq;
                    }
                }
                __syncthreads();
            }
    }
    if (t == 0) {
        int imin = 0;
        for (int i = 1; i < k; ++i)
            if (A[i][i] < A[imin][imin]) imin = i;
        red[0] = imin;
        const double theta = A[imin][imin];
        const double hlast = k == mm ? hd[(size_t)(mm - 1) * HESS_HC + 128] : 0.0;
        const double res = fabs(hlast * Z[k - 1][imin]);
        rec[0] = theta;
        rec[1] = theta != 0.0 ? res / fabs(theta) : res;
        rec[2] += k;
        rec[3] = k;
    }
    __syncthreads();
    const int imin = (int)red[0];
    if (t < mm) y[t] = t < k ? Z[t][imin] : 0.0;
}

void lanczos_eig(const double* hd, int mm, double* y, double* rec, hipStream_t s) {
    if (mm < 1 || mm > HESS_KMAX) ITE_FAIL(ITE_EINVAL, "lanczos_eig: Krylov dimension outside 1..64");
    hipLaunchKernelGGL(lanczos_eig_kernel, dim3(1), dim3(64), 0, s, hd, mm, y, rec);
    HIP_CHECK(hipGetLastError());
}

void hess_solve(const double* hd, int mm, double* y, double* stats, bool r_product, bool last_cycle, hipStream_t s) {
    if (mm < 1 || mm > HESS_KMAX) ITE_FAIL(ITE_EINVAL, "hess_solve: Krylov dimension outside 1..64");
    hipLaunchKernelGGL(hess_solve_kernel, dim3(1), dim3(64), 0, s, hd, mm, y, stats, (int)r_product, (int)last_cycle);
    HIP_CHECK(hipGetLastError());
}

void scale(double* x, double a, size_t n, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(scale_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, x, a, n);
    HIP_CHECK(hipGetLastError());
}

void fill(double* x, double v, size_t n, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, x, v, n);
    HIP_CHECK(hipGetLastError());
}

void eye(double* x, int D, hipStream_t s) {
    hipLaunchKernelGGL(eye_kernel, dim3(grid_for((size_t)D * D, 256)), dim3(256), 0, s, x, D);
    HIP_CHECK(hipGetLastError());
}

void nonfinite_any(const double* x, size_t n, int* flag, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(nonfinite_kernel, dim3(grid_for(n, 256, 1024)), dim3(256), 0, s, x, n, flag);
    HIP_CHECK(hipGetLastError());
}

void convert_f32(const double* x, float* y, size_t n, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(f32_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, x, y, n);
    HIP_CHECK(hipGetLastError());
}

void convert_bf16(const double* x, uint16_t* y, size_t n, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(bf16_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, x, y, n);
    HIP_CHECK(hipGetLastError());
}

void transpose(const double* in, int rows, int cols, double* out, hipStream_t s) {
    if (rows <= 0 || cols <= 0) return;
    dim3 grid((cols + 31) / 32, (rows + 31) / 32);
    hipLaunchKernelGGL(transpose_kernel, grid, dim3(32, 8), 0, s, in, rows, cols, out);
    HIP_CHECK(hipGetLastError());
}

template <int SC>
static void stage_launch(Stage st, hipStream_t s) {
    dim3 grid((st.C + SC - 1) / SC, st.G);
    size_t lds = (size_t)st.I * SC * sizeof(double);
    const size_t csr = (size_t)st.nnz * 12 + (size_t)(st.O + 1) * 4;
    st.csr_lds = st.nnz >= 0 && lds + csr <= STAGE_LDS_TOTAL;
    if (st.csr_lds) lds += csr;
    if (st.out_prec == 0) hipLaunchKernelGGL((stage_kernel<0, SC>), grid, dim3(SC), lds, s, st);
    else if (st.out_prec == 1) hipLaunchKernelGGL((stage_kernel<1, SC>), grid, dim3(SC), lds, s, st);
    else hipLaunchKernelGGL((stage_kernel<2, SC>), grid, dim3(SC), lds, s, st);
    HIP_CHECK(hipGetLastError());
}

// Whether the four-column kernel applies: unit column strides, strides and
// the column count multiples of 4, 16-byte aligned bases.
static bool stage4_ok(const Stage& st) {
    auto m4 = [](long v) { return v % 4 == 0; };
    auto al = [](const void* p, uintptr_t a) { return ((uintptr_t)p & (a - 1)) == 0; };
    if (st.in_cs != 1 || st.out_cs != 1 || st.C % 4 != 0) return false;
    if (!m4(st.in_gs) || !m4(st.in_s1) || (st.in_div > 1 && !m4(st.in_s2))) return false;
    if (!m4(st.out_gs) || !m4(st.out_s1) || (st.out_div > 1 && !m4(st.out_s2))) return false;
    const void* in = st.in_f32 ? static_cast<const void*>(st.in_f32) : static_cast<const void*>(st.in);
    if (!al(in, 16)) return false;
    if (st.out_prec == 0) return al(st.out, 16);
    return al(st.out_lo, st.out_prec == 1 ? 16 : 8);
}

template <int SC, typename TIN>
static void stage4_launch(Stage st, hipStream_t s) {
    dim3 grid((st.C / 4 + SC - 1) / SC, st.G);
    size_t lds = (size_t)st.I * 4 * SC * sizeof(TIN);
    lds = (lds + 7) & ~(size_t)7;
    const size_t csr = (size_t)st.nnz * 12 + (size_t)(st.O + 1) * 4;
    st.csr_lds = st.nnz >= 0 && lds + csr <= STAGE_LDS_TOTAL;
    if (st.csr_lds) lds += csr;
    if (st.out_prec == 0) hipLaunchKernelGGL((stage4_kernel<0, SC, TIN>), grid, dim3(SC), lds, s, st);
    else if (st.out_prec == 1) hipLaunchKernelGGL((stage4_kernel<1, SC, TIN>), grid, dim3(SC), lds, s, st);
    else hipLaunchKernelGGL((stage4_kernel<2, SC, TIN>), grid, dim3(SC), lds, s, st);
    HIP_CHECK(hipGetLastError());
}

template <typename TIN>
static void stage4_pick(const Stage& st, hipStream_t s) {
    const size_t per_col = (size_t)st.I * 4 * sizeof(TIN);
    if (per_col * 64 <= STAGE_LDS) stage4_launch<64, TIN>(st, s);
    else stage4_launch<32, TIN>(st, s);
}

void stage_f64(const Stage& st, hipStream_t s) {
    if (st.G <= 0 || st.C <= 0 || st.O <= 0) return;
    if (st.I < 1 || (size_t)st.I * 16 * sizeof(double) > STAGE_LDS)
        ITE_FAIL(ITE_EINVAL, "MPO stage: more than 1024 inputs per column");
    const size_t in_bytes = st.in_f32 ? sizeof(float) : sizeof(double);
    if (stage4_ok(st) && (size_t)st.I * 4 * 32 * in_bytes <= STAGE_LDS) {
        if (st.in_f32) stage4_pick<float>(st, s);
        else stage4_pick<double>(st, s);
        return;
    }
    const size_t per_col = (size_t)st.I * sizeof(double);
    if (per_col * 128 <= STAGE_LDS) stage_launch<128>(st, s);
    else if (per_col * 64 <= STAGE_LDS) stage_launch<64>(st, s);
    else if (per_col * 32 <= STAGE_LDS) stage_launch<32>(st, s);
    else stage_launch<16>(st, s);
}

// ---------------------------------------------------------------------------
// Batched fixed-budget GMRES (see BatchVec in internal.h)
// ---------------------------------------------------------------------------
namespace {

// Problem of unit u in a range split by the per-problem first units
// (start(g) increasing; G small): the last g with start(g) <= u.
template <typename F>
__device__ inline int unit_problem(int u, int G, F start) {
    int g = 0;
    while (g + 1 < G && start(g + 1) <= u) ++g;
    return g;
}

template <int KMAX>
__global__ __launch_bounds__(RT) void batch_reduce_kernel(const BatchVec* __restrict__ d, int G,
                                                          const int* __restrict__ tot, int mode, int k1) {
    __shared__ double sh[RT / 64];
    const int total = tot[BT_RED];
    for (int u = blockIdx.x; u < total; u += gridDim.x) {
        const int g = unit_problem(u, G, [&](int q) { return d[q].red_start; });
        const BatchVec& p = d[g];
        const int vb = u - p.red_start;
        if (vb >= p.nb) continue;
        if (mode <= 1 && p.small) continue;
        if (mode == 0) {
            mdot_block<KMAX>(p.V, p.n, k1, p.w, p.n, vb, p.nb, p.part, sh);
        } else {
            const double* x = mode == 1 ? p.w : (mode == 2 ? p.V : p.b);
            dot_block(x, x, p.n, vb, p.nb, p.part + vb, sh);
        }
    }
}

__global__ __launch_bounds__(RT) void batch_finish_kernel(const BatchVec* __restrict__ d, int G, int k, int k1,
                                                          int target) {
    __shared__ double sh[RT / 64];
    const int total = G * k1;
    for (int u = blockIdx.x; u < total; u += gridDim.x) {
        const int g = u / k1, j = u % k1;
        const BatchVec& p = d[g];
        if (target <= 2 && p.small) continue;
        double* col = p.hd + (size_t)k * HESS_HC;
        double* out;
        int mode = 2;
        if (target == 0) { out = col + j; mode = 0; }
        else if (target == 1) { out = col + 64 + j; mode = 0; }
        else if (target == 2) out = col + 128;
        else out = p.hd + (size_t)k * HESS_HC + (target == 3 ? 0 : 1);   // k = mm here: ||b||, ||r0||
        finish_one(p.part + (size_t)j * p.nb, p.nb, out, mode, sh);
    }
}

// w -= sum_(j < k1) c_j V_j, in chunks of 16 basis vectors as gemv_launch does.
__device__ inline double gemv_elem(const double* __restrict__ V, long ldv, int k1, const double* __restrict__ c,
                                   double wi, size_t i, bool sub) {
    for (int j0 = 0; j0 < k1; j0 += 16) {
        const int kk = k1 - j0 < 16 ? k1 - j0 : 16;
        double s = 0.0;
        for (int j = 0; j < kk; ++j) s += c[j0 + j] * V[(size_t)(j0 + j) * ldv + i];
        wi = sub ? wi - s : wi + s;
    }
    return wi;
}

__global__ __launch_bounds__(RT) void batch_vec_kernel(const BatchVec* __restrict__ d, int G,
                                                       const int* __restrict__ tot, int op, int k) {
    const int total = tot[BT_EW];
    for (int u = blockIdx.x; u < total; u += gridDim.x) {
        const int g = unit_problem(u, G, [&](int q) { return d[q].ew_start; });
        const BatchVec& p = d[g];
        if (op <= 2 && p.small) continue;
        const size_t i0 = (size_t)(u - p.ew_start) * BATCH_EW;
        const size_t i1 = min((size_t)p.n, i0 + BATCH_EW);
        const double* col = p.hd + (size_t)k * HESS_HC;
        if (op == 0 || op == 1) {
            const double* cf = op == 0 ? col : col + 64;
            for (size_t i = i0 + threadIdx.x; i < i1; i += RT) p.w[i] = gemv_elem(p.V, p.n, k + 1, cf, p.w[i], i, true);
        } else if (op == 2) {
            const double dd = col[128];
            const double inv = dd > 0.0 ? 1.0 / dd : 0.0;
            double* vn = p.V + (size_t)(k + 1) * p.n;
            for (size_t i = i0 + threadIdx.x; i < i1; i += RT) vn[i] = p.w[i] * inv;
        } else if (op == 3) {
            for (size_t i = i0 + threadIdx.x; i < i1; i += RT) p.V[i] = 1.0 * p.b[i] + -1.0 * p.V[i];
        } else if (op == 4) {
            const double dd = p.hd[(size_t)k * HESS_HC + 1];
            const double inv = dd > 0.0 ? 1.0 / dd : 0.0;
            for (size_t i = i0 + threadIdx.x; i < i1; i += RT) p.V[i] = p.V[i] * inv;
        } else if (op == 6) {
            const double* vk = p.V + (size_t)k * p.n;
            for (size_t i = i0 + threadIdx.x; i < i1; i += RT) p.tlo[i] = (float)vk[i];
        } else {
            for (size_t i = i0 + threadIdx.x; i < i1; i += RT) p.x[i] = gemv_elem(p.V, p.n, k, p.y, p.x[i], i, false);
        }
    }
}

template <int KMAX>
__global__ __launch_bounds__(CGS_T) void batch_cgs2_small_kernel(const BatchVec* __restrict__ d, int G, int k,
                                                                 int mm) {
    __shared__ CgsLDS<KMAX> sh;
    for (int g = blockIdx.x; g < G; g += gridDim.x) {
        const BatchVec& p = d[g];
        if (!p.small) continue;
        double* vnext = k + 1 < mm ? p.V + (size_t)(k + 1) * p.n : nullptr;
        cgs2_small_body<KMAX>(p.V, p.n, k + 1, p.w, (int)p.n, p.hd + (size_t)k * HESS_HC, vnext, sh);
        __syncthreads();
    }
}

__global__ __launch_bounds__(64) void batch_hess_kernel(const BatchVec* __restrict__ d, int G, int mm, int r_product,
                                                        int last_cycle) {
    __shared__ double Hs[HESS_LDS];
    for (int g = blockIdx.x; g < G; g += gridDim.x) {
        const BatchVec& p = d[g];
        if (threadIdx.x == 0) hess_solve_one(p.hd, mm, p.y, p.stats, r_product, last_cycle, Hs);
        __syncthreads();
    }
}

// LO: the FP32 stage st_lo (FP32 output) instead of st.
template <bool LO>
__global__ __launch_bounds__(BATCH_STAGE_SC) void batch_stage_kernel(const BatchVec* __restrict__ d, int G,
                                                                     const int* __restrict__ tot) {
    __shared__ double xin[BATCH_STAGE_SC * BATCH_STAGE_SC];
    const int total = tot[BT_STAGE];
    for (int u = blockIdx.x; u < total; u += gridDim.x) {
        const int g = unit_problem(u, G, [&](int q) { return d[q].stage_start; });
        const Stage& st = LO ? d[g].st_lo : d[g].st;
        const int nc = (st.C + BATCH_STAGE_SC - 1) / BATCH_STAGE_SC;
        const int lu = u - d[g].stage_start;
        stage_unit<LO ? 1 : 0, BATCH_STAGE_SC>(st, lu / nc, lu % nc, xin);
    }
}

__global__ __launch_bounds__(64) void batch_zero_stats_kernel(const BatchVec* __restrict__ d, int G) {
    for (int g = blockIdx.x; g < G; g += gridDim.x)
        if (threadIdx.x < 8) d[g].stats[threadIdx.x] = 0.0;
}

}  // namespace

void batch_zero_stats(const BatchVec* d, int G, hipStream_t s) {
    if (G <= 0) return;
    hipLaunchKernelGGL(batch_zero_stats_kernel, dim3(std::min(G, BATCH_GRID)), dim3(64), 0, s, d, G);
    HIP_CHECK(hipGetLastError());
}

void batch_reduce(const BatchVec* d, int G, const int* tot, int mode, int k1, hipStream_t s) {
    if (G <= 0) return;
    if (mode == 0 && k1 > 16) ITE_FAIL(ITE_EINVAL, "batch_reduce: at most 16 basis vectors per launch");
    if (mode != 0 || k1 <= 4)
        hipLaunchKernelGGL((batch_reduce_kernel<4>), dim3(BATCH_GRID), dim3(RT), 0, s, d, G, tot, mode, k1);
    else if (k1 <= 8)
        hipLaunchKernelGGL((batch_reduce_kernel<8>), dim3(BATCH_GRID), dim3(RT), 0, s, d, G, tot, mode, k1);
    else
        hipLaunchKernelGGL((batch_reduce_kernel<16>), dim3(BATCH_GRID), dim3(RT), 0, s, d, G, tot, mode, k1);
    HIP_CHECK(hipGetLastError());
}

void batch_finish(const BatchVec* d, int G, int k, int k1, int target, hipStream_t s) {
    if (G <= 0) return;
    hipLaunchKernelGGL(batch_finish_kernel, dim3(std::min(BATCH_GRID, G * k1)), dim3(RT), 0, s, d, G, k, k1, target);
    HIP_CHECK(hipGetLastError());
}

void batch_vec(const BatchVec* d, int G, const int* tot, int op, int k, hipStream_t s) {
    if (G <= 0) return;
    hipLaunchKernelGGL(batch_vec_kernel, dim3(BATCH_GRID), dim3(RT), 0, s, d, G, tot, op, k);
    HIP_CHECK(hipGetLastError());
}

void batch_cgs2_small(const BatchVec* d, int G, int k, int mm, hipStream_t s) {
    if (G <= 0) return;
    const int k1 = k + 1;
    const dim3 grid(std::min(G, BATCH_GRID));
    if (k1 <= 8) hipLaunchKernelGGL((batch_cgs2_small_kernel<8>), grid, dim3(CGS_T), 0, s, d, G, k, mm);
    else if (k1 <= 16) hipLaunchKernelGGL((batch_cgs2_small_kernel<16>), grid, dim3(CGS_T), 0, s, d, G, k, mm);
    else if (k1 <= 32) hipLaunchKernelGGL((batch_cgs2_small_kernel<32>), grid, dim3(CGS_T), 0, s, d, G, k, mm);
    else hipLaunchKernelGGL((batch_cgs2_small_kernel<64>), grid, dim3(CGS_T), 0, s, d, G, k, mm);
    HIP_CHECK(hipGetLastError());
}

void batch_hess(const BatchVec* d, int G, int mm, bool r_product, bool last_cycle, hipStream_t s) {
    if (G <= 0) return;
    if (mm < 1 || mm > HESS_KMAX) ITE_FAIL(ITE_EINVAL, "batch_hess: Krylov dimension outside 1..64");
    hipLaunchKernelGGL(batch_hess_kernel, dim3(std::min(G, BATCH_GRID)), dim3(64), 0, s, d, G, mm, (int)r_product,
                       (int)last_cycle);
    HIP_CHECK(hipGetLastError());
}

void batch_stage(const BatchVec* d, int G, const int* tot, hipStream_t s) {
    if (G <= 0) return;
    hipLaunchKernelGGL(batch_stage_kernel<false>, dim3(BATCH_GRID), dim3(BATCH_STAGE_SC), 0, s, d, G, tot);
    HIP_CHECK(hipGetLastError());
}

void batch_stage_lo(const BatchVec* d, int G, const int* tot, hipStream_t s) {
    if (G <= 0) return;
    hipLaunchKernelGGL(batch_stage_kernel<true>, dim3(BATCH_GRID), dim3(BATCH_STAGE_SC), 0, s, d, G, tot);
    HIP_CHECK(hipGetLastError());
}

}  // namespace ite
