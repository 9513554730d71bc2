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
// columns are updated as Z_t <- Z_t - V (T^T (V^T Z_t)) by one launch whose
// workgroups own 16-column blocks (FP64 MFMA).
// The reflectors are kept transposed (one row per reflector) so that they are
// written and read in whole rows.
#include "internal.h"
#include "wave.h"

#include <algorithm>

namespace ite {
namespace {

constexpr int QB = 16;        // panel width
constexpr int QRPL = 32;      // panel rows per lane: panels of up to 64 * 32 = 2048 rows

// Factor the m x nbw panel at P (leading dimension ld), nbw <= QB, m <= 2048.
// Writes R (upper triangle) and zeros below it into the panel, the reflectors
// transposed to VT [QB][m] (row j = reflector j: zero above row j, one at row
// j; rows nbw..QB-1 zero) and T [QB][QB] (upper triangular).  The panel moves
// between memory and the wavefronts' registers through LDS in chunks of
// QCH rows, so that every global access reads or writes whole rows.  Eight
// wavefronts, wavefront w owning columns w and w + 8 (each lane 32 rows of
// both); a column keeps its reflector in its registers below the diagonal
// (where R is zero).  Per reflector the owning wavefront writes it to LDS
// once and every wavefront reads it once into registers, then applies it to
// its columns right of j or, left of j, forms their entries v_i . v_j of
// S = V^T V, which the recursion for T needs.
constexpr int QCH = 512;
constexpr int QNC = 64 * QRPL / QCH;    // LDS chunks per panel
constexpr int QPW = 8;                  // wavefronts of the panel kernel

// Reflector j from the column held in a (LAPACK's convention:
// beta = -sign(alpha) ||x||, tau = (beta - alpha) / beta,
// v = x / (alpha - beta) with v_j = 1; tau = 0 when x_(j+1..) = 0); v goes
// to vs (all 64 QRPL rows), beta and v replace the column from row j on.
// Rows at and past m hold zeros, and j < QB <= 64: only the rows of a[0]
// need comparing with j.
__device__ __forceinline__ void qr_reflector(double (&a)[QRPL], int j, int lane, double* vs, double* tau_s,
                                             double (*S)[QB + 1]) {
    const double alpha = lane_value(a[0], j);     // row j < QB lies in a[0] of lane j
    double sg = lane > j ? a[0] * a[0] : 0.0;
#pragma unroll
    for (int i = 1; i < QRPL; ++i) sg += a[i] * a[i];
    sg = wave_sum(sg);
    double tau = 0.0, beta = alpha, scale = 0.0;
    if (sg > 0.0) {
        const double nrm = sqrt(alpha * alpha + sg);
        beta = alpha >= 0.0 ? -nrm : nrm;
        tau = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
    }
    {
        const double v = lane == j ? 1.0 : (lane > j ? a[0] * scale : 0.0);
        vs[lane] = v;
        a[0] = lane < j ? a[0] : (lane == j ? beta : v);
    }
#pragma unroll
    for (int i = 1; i < QRPL; ++i) {
        a[i] *= scale;
        vs[lane + 64 * i] = a[i];
    }
    if (lane == 0) {
        tau_s[j] = tau;
        S[j][j] = 1.0 + sg * scale * scale;    // v . v
    }
}

// Reflector j (v, in registers) on column c held in a: for c > j the
// update a -= tau v (v . a); for c < j the entry S[c][j] = v_c . v_j.
__device__ __forceinline__ void qr_column_step(double (&a)[QRPL], const double (&v)[QRPL], int c, int j, int nbw,
                                               int lane, double tau, double (*S)[QB + 1]) {
    if (c >= nbw || c == j) return;
    // column c's values (c > j) or its reflector (c < j: one at row c, zero
    // above it) against v; rows of a[1..] lie below every row < QB
    double dot = v[0] * (c > j ? a[0] : (lane == c ? 1.0 : (lane > c ? a[0] : 0.0)));
#pragma unroll
    for (int i = 1; i < QRPL; ++i) dot += v[i] * a[i];
    dot = wave_sum(dot);
    if (c > j) {
        const double f = tau * dot;
#pragma unroll
        for (int i = 0; i < QRPL; ++i) a[i] -= f * v[i];
    } else if (lane == 0) {
        S[c][j] = dot;
    }
}

__global__ __launch_bounds__(64 * QPW) void qr_panel_kernel(double* __restrict__ P, int ld, int m, int nbw,
                                                            double* __restrict__ VT, double* __restrict__ T) {
    constexpr int NT = 64 * QPW;
    __shared__ double Pc[QCH][QB + 1];
    __shared__ double vs[2][64 * QRPL];   // reflectors j (buffer j mod 2)
    __shared__ double tau_s[QB];
    __shared__ double S[QB][QB + 1];
    __shared__ double Ts[QB][QB + 1];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int c0 = w, c1 = w + QPW;               // this wavefront's columns
    if (t < QB * (QB + 1)) S[t / (QB + 1)][t % (QB + 1)] = 0.0;
    double a0[QRPL], a1[QRPL];
    // coalesced load through LDS: QB consecutive lanes move one row of the
    // chunk (one load touches NT / QB rows, not one row per lane)
    static_assert((QCH * QB) % NT == 0 && NT % QB == 0, "chunk layout");
    constexpr int LPT = QCH * QB / NT;
    const int er = t % QB, rr0 = t / QB;
#pragma unroll
    for (int c = 0; c < QNC; ++c) {
        {
            double ldv[LPT];
#pragma unroll
            for (int h = 0; h < LPT; ++h) {
                const int row = c * QCH + rr0 + h * (NT / QB);
                ldv[h] = (row < m && er < nbw) ? P[(long)row * ld + er] : 0.0;
            }
#pragma unroll
            for (int h = 0; h < LPT; ++h) Pc[rr0 + h * (NT / QB)][er] = ldv[h];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < QRPL; ++i) {
            if (64 * i < c * QCH || 64 * i >= (c + 1) * QCH) continue;
            const int r = lane + 64 * i - c * QCH;
            a0[i] = Pc[r][c0];
            a1[i] = Pc[r][c1];
        }
        __syncthreads();
    }
    // Look-ahead: after applying reflector j to its columns, the owner of
    // column j + 1 forms reflector j + 1 into the other buffer before the
    // barrier, so one barrier per column separates the reflectors (each
    // column still sees the reflectors in order: the same arithmetic as
    // without look-ahead).
    if (nbw > 0 && w == 0) qr_reflector(a0, 0, lane, vs[0], tau_s, S);
    __syncthreads();
    for (int j = 0; j < nbw; ++j) {
        const double* vj = vs[j & 1];
        for (int row = t; row < m; row += NT) VT[(long)j * m + row] = vj[row];
        double v[QRPL];
#pragma unroll
        for (int i = 0; i < QRPL; ++i) v[i] = vj[lane + 64 * i];
        const double tau = tau_s[j];
        qr_column_step(a0, v, c0, j, nbw, lane, tau, S);
        qr_column_step(a1, v, c1, j, nbw, lane, tau, S);
        const int jn = j + 1;
        if (jn < nbw && w == (jn & (QPW - 1))) {
            if (jn < QPW)
                qr_reflector(a0, jn, lane, vs[jn & 1], tau_s, S);
            else
                qr_reflector(a1, jn, lane, vs[jn & 1], tau_s, S);
        }
        __syncthreads();
    }
    // coalesced write-back of R and the zeros below it (the reflectors held
    // below the diagonal are not part of R)
#pragma unroll
    for (int c = 0; c < QNC; ++c) {
#pragma unroll
        for (int i = 0; i < QRPL; ++i) {
            if (64 * i < c * QCH || 64 * i >= (c + 1) * QCH) continue;
            const int row = lane + 64 * i;
            Pc[row - c * QCH][c0] = row > c0 ? 0.0 : a0[i];
            Pc[row - c * QCH][c1] = row > c1 ? 0.0 : a1[i];
        }
        __syncthreads();
#pragma unroll
        for (int h = 0; h < LPT; ++h) {
            const int row = c * QCH + rr0 + h * (NT / QB);
            if (row < m && er < nbw) P[(long)row * ld + er] = Pc[rr0 + h * (NT / QB)][er];
        }
        __syncthreads();
    }
    // reflector rows nbw..QB-1 are zero
    for (int e = t; e < (QB - nbw) * m; e += NT) VT[(long)nbw * m + e] = 0.0;
    if (t < QB && t >= nbw) tau_s[t] = 0.0;
    __syncthreads();
    // T: T_jj = tau_j, T[0:j, j] = -tau_j T[0:j, 0:j] S[0:j, j]; lane i of
    // the first wavefront holds row i of T in registers (entries left of the
    // diagonal are zero, so the sum over k < j equals the one over i <= k < j)
    if (t < 64) {
        const int i = t;
        double trow[QB];
#pragma unroll
        for (int j = 0; j < QB; ++j) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < j; ++k) acc += trow[k] * S[k][j];
            trow[j] = i < j ? -tau_s[j] * acc : (i == j ? tau_s[j] : 0.0);
        }
        if (i < QB) {
#pragma unroll
            for (int j = 0; j < QB; ++j) Ts[i][j] = trow[j];
        }
    }
    __syncthreads();
    if (t < QB * QB) T[t] = Ts[t / QB][t % QB];
}

typedef double d4_t __attribute__((ext_vector_type(4)));

// Zt[:, cbeg:cbeg + 16 NCT] <- (I - V T V^T)^T Zt = Zt - V (T^T (V^T Zt)) for
// the reflectors VT [QB][m] and T [QB][QB], by one workgroup of 16
// wavefronts, in one pass over the rows for W = V^T Zt (FP64 MFMA, the rows
// split over the wavefronts, partials summed in LDS) and one for the update
// (FP64 MFMA, K = QB).  Columns at and past cend are left alone.
template <int NCT>
__global__ __launch_bounds__(1024) void qr_apply_kernel(double* __restrict__ Zt, int ld, int m, int nt,
                                                        const double* __restrict__ VT,
                                                        const double* __restrict__ T) {
    constexpr int CW = 16 * NCT;
    __shared__ double Wp[16][QB][CW + 1];
    __shared__ double W2[QB][CW + 1];
    __shared__ double Ts[QB][QB + 1];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int l16 = lane & 15, kg = lane >> 4;
    const int cbeg = blockIdx.x * CW, cend = min(nt, cbeg + CW);
    if (t < QB * QB) Ts[t / QB][t % QB] = T[t];
    // W partials: wavefront w sums over its slice of rows
    {
        const int rw = ((m + 15) / 16 + 3) & ~3;
        const int r0 = w * rw, r1 = min(m, r0 + rw);
        d4_t acc[NCT];
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) acc[ct] = d4_t{0, 0, 0, 0};
        // four k steps per iteration, their loads issued together
        for (int k0 = r0; k0 < r1; k0 += 16) {
            double av[4], bv[4][NCT];
#pragma unroll
            for (int st = 0; st < 4; ++st) {
                const int row = k0 + 4 * st + kg;
                av[st] = row < r1 ? VT[(long)l16 * m + row] : 0.0;
#pragma unroll
                for (int ct = 0; ct < NCT; ++ct) {
                    const int col = cbeg + ct * 16 + l16;
                    bv[st][ct] = (row < r1 && col < cend) ? Zt[(long)row * ld + col] : 0.0;
                }
            }
#pragma unroll
            for (int st = 0; st < 4; ++st)
#pragma unroll
                for (int ct = 0; ct < NCT; ++ct)
                    acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[st], bv[st][ct], acc[ct], 0, 0, 0);
        }
        // FP64 MFMA accumulator element rr of lane group kg is row 4 rr + kg
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) Wp[w][4 * rr + kg][ct * 16 + l16] = acc[ct][rr];
    }
    __syncthreads();
    // W2 = T^T W, negated for the update below
    if (t < QB * CW) {
        const int i = t / CW, c = t % CW;
        double sw = 0.0;
        for (int ww = 0; ww < 16; ++ww) sw += Wp[ww][i][c];
        Wp[0][i][c] = sw;     // row i of W; only this thread reads it back
    }
    __syncthreads();
    if (t < QB * CW) {
        const int r = t / CW, c = t % CW;
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < QB; ++k) acc += Ts[k][r] * Wp[0][k][c];
        W2[r][c] = -acc;
    }
    __syncthreads();
    // Zt -= V W2: 16-row tiles over the wavefronts
    const int nrt = (m + 15) / 16;
    for (int rt = w; rt < nrt; rt += 16) {
        const int rowa = rt * 16 + l16;            // A operand row (V row)
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
            const int col = cbeg + ct * 16 + l16;
            d4_t acc;
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const int row = rt * 16 + 4 * rr + kg;
                acc[rr] = (row < m && col < cend) ? Zt[(long)row * ld + col] : 0.0;
            }
#pragma unroll
            for (int ks = 0; ks < QB / 4; ++ks) {
                const int k = 4 * ks + kg;
                const double a = rowa < m ? VT[(long)k * m + rowa] : 0.0;
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, W2[k][ct * 16 + l16], acc, 0, 0, 0);
            }
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const int row = rt * 16 + 4 * rr + kg;
                if (row < m && col < cend) Zt[(long)row * ld + col] = acc[rr];
            }
        }
    }
}

constexpr int QNCT = 1;       // column tiles per apply workgroup

}  // namespace

bool householder_applies(int p, int q) { return p >= 256 && p <= 64 * QRPL && q >= QB; }

size_t householder_workspace(int p, int q, int ld) {
    (void)q;
    (void)ld;
    return (size_t)p * QB + QB * QB + 256;
}

void householder_rows(double* Z, int p, int q, int ld, double* ws, hipStream_t s) {
    const int kmax = std::min(p, q);
    double* VT = ws;
    double* T = VT + (size_t)p * QB;
    for (int c0 = 0; c0 < kmax; c0 += QB) {
        const int nbw = std::min(QB, kmax - c0);
        const int m = p - c0;
        double* P = Z + (long)c0 * ld + c0;
        hipLaunchKernelGGL(qr_panel_kernel, dim3(1), dim3(64 * QPW), 0, s, P, ld, m, nbw, VT, T);
        const int nt = ld - (c0 + nbw);
        if (nt <= 0) continue;
        constexpr int CW = 16 * QNCT;
        hipLaunchKernelGGL((qr_apply_kernel<QNCT>), dim3((nt + CW - 1) / CW), dim3(1024), 0, s, P + nbw, ld, m, nt,
                           VT, T);
    }
    HIP_CHECK(hipGetLastError());
}

}  // namespace ite
