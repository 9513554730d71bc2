// Householder QR preconditioning of the one-sided Jacobi split.
//
// The Jacobi work matrix Z = [X | I] (p rows) is replaced by Q^T Z, where
// X = Q R is the Householder QR of X: the rows of the first part become the
// rows of R, and the second part becomes Q^T.  An orthogonal transform of the
// rows changes nothing the one-sided Jacobi computes (it ends at the same
// [Sigma V^T | U^T] up to the choice of basis within equal singular values),
// but the rows of R are graded like the singular values, and on such rows
// the Jacobi sweeps converge in far fewer sweeps (Drmac and Veselic's
// preconditioned Jacobi).  When p > q the rows q..p-1 of R vanish and the
// Jacobi only needs the first q rows; their Q^T part completes the basis.
//
// Blocked Householder with the compact WY form (Schreiber and Van Loan):
// per panel of QB columns, one workgroup factors the panel (wavefront j owns
// column j, each lane 32 of its rows), writes the reflectors V and the
// triangular factor T with H_1 ... H_QB = I - V T V^T, and the trailing
// columns are updated as Z_t <- Z_t - V (T^T (V^T Z_t)) with FP64 MFMA GEMMs.
// The reflectors are kept transposed (one row per reflector) so that they are
// written and read in whole rows.
#include "internal.h"

#include <algorithm>

namespace ite {
namespace {

constexpr int QB = 16;        // panel width
constexpr int QRPL = 32;      // panel rows per lane: panels of up to 64 * 32 = 2048 rows
constexpr int QKC = 128;      // rows per K chunk of V^T Z_t
typedef double d4_t __attribute__((ext_vector_type(4)));

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Factor the m x nbw panel at P (leading dimension ld), nbw <= QB, m <= 2048.
// Writes R (upper triangle) and zeros below it into the panel, the reflectors
// transposed to VT [QB][m] (row j = reflector j: zero above row j, one at row
// j; rows nbw..QB-1 zero) and T [QB][QB] (upper triangular).  The panel moves
// between memory and the wavefronts' registers through LDS in chunks of
// QCH rows, so that every global access reads or writes whole rows.
constexpr int QCH = 512;
__global__ __launch_bounds__(1024) void qr_panel_kernel(double* __restrict__ P, int ld, int m, int nbw,
                                                        double* __restrict__ VT, double* __restrict__ T) {
    __shared__ double Pc[QCH][QB + 1];
    __shared__ double vs[64 * QRPL];
    __shared__ double tau_s[QB];
    __shared__ double Sp[16][QB][QB + 1];
    __shared__ double S[QB][QB + 1];
    __shared__ double Ts[QB][QB + 1];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const bool own = w < nbw;
    double a[QRPL];
#pragma unroll
    for (int i = 0; i < QRPL; ++i) a[i] = 0.0;
    // coalesced load: thread t moves 8 consecutive entries of row t / 2
    for (int c0 = 0; c0 < 64 * QRPL; c0 += QCH) {
        {
            const int rr = t >> 1, h = (t & 1) * 8;
            const int row = c0 + rr;
#pragma unroll
            for (int e = 0; e < 8; ++e)
                Pc[rr][h + e] = (row < m && h + e < nbw) ? P[(long)row * ld + h + e] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < QRPL; ++i) {
            const int row = lane + 64 * i;
            if (row >= c0 && row < c0 + QCH) a[i] = Pc[row - c0][w];
        }
        __syncthreads();
    }
    for (int j = 0; j < nbw; ++j) {
        if (w == j) {
            // reflector of column j over rows j..m-1 (LAPACK's convention:
            // beta = -sign(alpha) ||x||, tau = (beta - alpha) / beta,
            // v = x / (alpha - beta) with v_j = 1; tau = 0 when x_(j+1..) = 0)
            const double alpha = __shfl(a[0], j, 64);     // row j < QB lies in a[0] of lane j
            double sg = 0.0;
#pragma unroll
            for (int i = 0; i < QRPL; ++i) {
                const int row = lane + 64 * i;
                if (row > j && row < m) sg += a[i] * a[i];
            }
            sg = wave_sum(sg);
            double tau = 0.0, beta = alpha, scale = 0.0;
            if (sg > 0.0) {
                const double nrm = sqrt(alpha * alpha + sg);
                beta = alpha >= 0.0 ? -nrm : nrm;
                tau = (beta - alpha) / beta;
                scale = 1.0 / (alpha - beta);
            }
#pragma unroll
            for (int i = 0; i < QRPL; ++i) {
                const int row = lane + 64 * i;
                const double v = row == j ? 1.0 : ((row > j && row < m) ? a[i] * scale : 0.0);
                vs[row] = v;
                a[i] = row < j ? a[i] : (row == j ? beta : 0.0);
            }
            if (lane == 0) tau_s[j] = tau;
        }
        __syncthreads();
        for (int row = t; row < m; row += 1024) VT[(long)j * m + row] = vs[row];
        if (own && w > j) {
            const double tau = tau_s[j];
            double dot = 0.0;
#pragma unroll
            for (int i = 0; i < QRPL; ++i) dot += vs[lane + 64 * i] * a[i];
            const double f = tau * wave_sum(dot);
            // reload v from LDS below rather than keeping 32 more values live
            asm volatile("" ::: "memory");
#pragma unroll
            for (int i = 0; i < QRPL; ++i) a[i] -= f * vs[lane + 64 * i];
        }
        __syncthreads();
    }
    // coalesced write-back of R and the zeros below it
    for (int c0 = 0; c0 < 64 * QRPL; c0 += QCH) {
#pragma unroll
        for (int i = 0; i < QRPL; ++i) {
            const int row = lane + 64 * i;
            if (row >= c0 && row < c0 + QCH) Pc[row - c0][w] = a[i];
        }
        __syncthreads();
        {
            const int rr = t >> 1, h = (t & 1) * 8;
            const int row = c0 + rr;
#pragma unroll
            for (int e = 0; e < 8; ++e)
                if (row < m && h + e < nbw) P[(long)row * ld + h + e] = Pc[rr][h + e];
        }
        __syncthreads();
    }
    // reflector rows nbw..QB-1 are zero
    for (int e = t; e < (QB - nbw) * m; e += 1024) VT[(long)nbw * m + e] = 0.0;
    if (t < QB && t >= nbw) tau_s[t] = 0.0;
    __syncthreads();
    // S = V^T V with FP64 MFMA, the rows split over the 16 wavefronts
    {
        const int l16 = lane & 15, kg = lane >> 4;
        d4_t acc = {0, 0, 0, 0};
        const int rows_per_wave = (m + 15) / 16;
        const int r0 = w * rows_per_wave, r1 = min(m, r0 + rows_per_wave);
        for (int k0 = r0; k0 < r1; k0 += 4) {
            const int row = k0 + kg;
            const double v = (row < r1) ? VT[(long)l16 * m + row] : 0.0;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(v, v, acc, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) Sp[w][4 * r + kg][l16] = acc[r];
    }
    __syncthreads();
    if (t < QB * QB) {
        const int i = t / QB, k = t % QB;
        double s = 0.0;
        for (int ww = 0; ww < 16; ++ww) s += Sp[ww][i][k];
        S[i][k] = s;
    }
    __syncthreads();
    // T: T_jj = tau_j, T[0:j, j] = -tau_j T[0:j, 0:j] S[0:j, j]; column j by
    // lanes i < j of the first wavefront, one column after the other
    if (t < 64) {
        const int i = t;
        for (int j = 0; j < QB; ++j) {
            double tij = 0.0;
            if (i < j) {
                double acc = 0.0;
                for (int k = i; k < j; ++k) acc += Ts[i][k] * S[k][j];
                tij = -tau_s[j] * acc;
            } else if (i == j) {
                tij = tau_s[j];
            }
            if (i < QB) Ts[i][j] = tij;
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        }
    }
    __syncthreads();
    if (t < QB * QB) T[t] = Ts[t / QB][t % QB];
}

// W2[r][c] = sum_k T[k][r] W[k][c] with W = sum over nchunk partials
// Wp[b][k][c] (b < nchunk, k < QB, c < n).  Block: 16 rows x 64 columns.
__global__ __launch_bounds__(1024) void qr_reduce_t_kernel(const double* __restrict__ Wp, int nchunk, int n,
                                                           const double* __restrict__ T, double* __restrict__ W2) {
    __shared__ double Ws[QB][64 + 1];
    __shared__ double Ts[QB][QB + 1];
    const int t = threadIdx.x, r = t / 64, cl = t % 64;
    const int c = blockIdx.x * 64 + cl;
    if (t < QB * QB) Ts[t / QB][t % QB] = T[t];
    double s = 0.0;
    if (c < n)
        for (int b = 0; b < nchunk; ++b) s += Wp[((long)b * QB + r) * n + c];
    Ws[r][cl] = s;
    __syncthreads();
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < QB; ++k) acc += Ts[k][r] * Ws[k][cl];
    if (c < n) W2[(long)r * n + c] = acc;
}

}  // namespace

bool householder_applies(int p, int q) { return p >= 256 && p <= 64 * QRPL && q >= QB; }

size_t householder_workspace(int p, int q, int ld) {
    const int nt = ld;   // trailing columns are at most ld
    const int nchunk = (p + QKC - 1) / QKC;
    return (size_t)p * QB + QB * QB + (size_t)nchunk * QB * nt + (size_t)QB * nt + 256;
}

void householder_rows(double* Z, int p, int q, int ld, double* ws, hipStream_t s) {
    const int kmax = std::min(p, q);
    double* VT = ws;
    double* T = VT + (size_t)p * QB;
    double* Wp = T + QB * QB;
    const int nchunk_max = (p + QKC - 1) / QKC;
    double* W2 = Wp + (size_t)nchunk_max * QB * ld;
    for (int c0 = 0; c0 < kmax; c0 += QB) {
        const int nbw = std::min(QB, kmax - c0);
        const int m = p - c0;
        double* P = Z + (long)c0 * ld + c0;
        hipLaunchKernelGGL(qr_panel_kernel, dim3(1), dim3(1024), 0, s, P, ld, m, nbw, VT, T);
        const int nt = ld - (c0 + nbw);
        if (nt <= 0) continue;
        double* Zt = P + nbw;
        // Wp[b] = V[b-th chunk]^T Zt[b-th chunk]: full chunks in one batched
        // launch, the remainder in a second
        const int nfull = m / QKC, rem = m % QKC;
        if (nfull > 0) {
            Gemm g;
            g.M = QB; g.N = nt; g.K = QKC;
            g.A = VT; g.lda = m; g.sA = QKC;
            g.B = Zt; g.ldb = ld; g.sB = (long)QKC * ld;
            g.D = Wp; g.ldd = nt; g.sD = (long)QB * nt;
            g.batch = nfull;
            gemm_f64(g, s);
        }
        if (rem > 0) {
            Gemm g;
            g.M = QB; g.N = nt; g.K = rem;
            g.A = VT + (long)nfull * QKC; g.lda = m;
            g.B = Zt + (long)nfull * QKC * ld; g.ldb = ld;
            g.D = Wp + (long)nfull * QB * nt; g.ldd = nt;
            gemm_f64(g, s);
        }
        const int nchunk = nfull + (rem > 0 ? 1 : 0);
        hipLaunchKernelGGL(qr_reduce_t_kernel, dim3((nt + 63) / 64), dim3(1024), 0, s, Wp, nchunk, nt, T, W2);
        // Zt -= V W2 (V = VT^T)
        Gemm u;
        u.M = m; u.N = nt; u.K = QB; u.tA = true; u.alpha = -1.0; u.beta = 1.0;
        u.A = VT; u.lda = m;
        u.B = W2; u.ldb = nt;
        u.C = Zt; u.ldc = ld;
        u.D = Zt; u.ldd = ld;
        gemm_f64(u, s);
    }
    HIP_CHECK(hipGetLastError());
}

}  // namespace ite
