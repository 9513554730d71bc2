// One-sided (Hestenes) block-Jacobi SVD for the bond truncation of the
// two-site sweep (Heisenberg chain section: truncation by discarded weight;
// Appendix D: bond cap).
//
// The rows of the first q columns of a work matrix Z[p][ld] are made mutually
// orthogonal by orthogonal row rotations, and the same rotations are applied
// to all ld columns.  With Z = [X | I_p] the final rows are
// [sigma_i v_i^T | u_i^T] for X = U diag(sigma) V^T, so both factors come out
// of one run and the rotation part is a complete orthonormal basis even when
// some sigma_i are zero.
//
// Rows are grouped in blocks of 16; a round-robin (circle) schedule pairs the
// blocks so that every pair meets once per sweep.  For each pair of blocks
// (32 rows):
//   1. gram:   G = X_pair X_pair^T, summed over column chunks with FP64 MFMA;
//   2. inner:  G = Q diag Q^T by cyclic two-sided Jacobi on the 32 x 32
//              matrix in LDS (one wavefront); Q accumulates the rotations;
//   3. rotate: Z_pair <- Q^T Z_pair over all ld columns.
// Pairs whose rows are already orthogonal to the working tolerance produce no
// rotation and skip step 3.  A sweep ends with one host read of the largest
// relative off-diagonal |G_ij| / sqrt(G_ii G_jj) seen in it.
#include "internal.h"

#include <algorithm>
#include <cmath>

namespace ite {
namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));

constexpr int RB = 16;       // rows per block
constexpr int PR = 2 * RB;   // rows per pair
constexpr int GW = 128;      // columns per gram chunk
constexpr int RW = 256;      // columns per rotate block

// Block index at position `pos` of the circle schedule in round r
// (nb blocks, nb even; position 0 is fixed).
__device__ inline int circle_block(int pos, int r, int nb) {
    return pos == 0 ? 0 : ((pos - 1 + r) % (nb - 1)) + 1;
}

__device__ inline int pair_row(int P, int lr, int r, int nb) {
    const int bi = circle_block(P, r, nb);
    const int bj = circle_block(nb - 1 - P, r, nb);
    return lr < RB ? bi * RB + lr : bj * RB + (lr - RB);
}

__global__ __launch_bounds__(256) void gram_kernel(const double* __restrict__ Z, int p, int q,
                                                   int ld, int r, int nb, int nchunks,
                                                   double* __restrict__ gram) {
    __shared__ double Xs[PR][GW + 1];
    const int P = blockIdx.y, chunk = blockIdx.x;
    const int c0 = chunk * GW;
    const int t = threadIdx.x;
    for (int e = 0; e < PR / 2; ++e) {
        const int lr = 2 * e + (t >> 7);
        const int c = c0 + (t & 127);
        const int row = pair_row(P, lr, r, nb);
        Xs[lr][t & 127] = (row < p && c < q) ? Z[(long)row * ld + c] : 0.0;
    }
    __syncthreads();
    const int lane = t & 63, w = t >> 6;
    const int I = w >> 1, J = w & 1;
    const int l16 = lane & 15, kg = lane >> 4;
    d4_t acc = {0, 0, 0, 0};
    for (int k0 = 0; k0 < GW; k0 += 4)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Xs[I * 16 + l16][k0 + kg], Xs[J * 16 + l16][k0 + kg],
                                                   acc, 0, 0, 0);
    double* out = gram + ((long)P * nchunks + chunk) * (PR * PR);
    // FP64 MFMA accumulator element rr of lane group kg is tile row 4 rr + kg
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) out[(I * 16 + 4 * rr + kg) * PR + J * 16 + l16] = acc[rr];
}

__device__ inline void atomic_max_pos(double* addr, double v) {
    // non-negative doubles order like their bit patterns
    atomicMax(reinterpret_cast<unsigned long long*>(addr), (unsigned long long)__double_as_longlong(v));
}

// One wavefront per pair: sum the chunk partials, diagonalise by cyclic
// Jacobi, write Q (32 x 32) and whether any rotation was applied.
__global__ __launch_bounds__(64) void inner_kernel(const double* __restrict__ gram, int nchunks,
                                                   int p, int r, int nb, double tol,
                                                   int inner_sweeps, double* __restrict__ rot,
                                                   int* __restrict__ rotated,
                                                   double* __restrict__ sweep_off) {
    __shared__ double G[PR][PR + 1];
    __shared__ double Q[PR][PR + 1];
    __shared__ double cs[PR / 2], sn[PR / 2];
    __shared__ int pa[PR / 2], pb[PR / 2];
    __shared__ int any_rot;
    const int P = blockIdx.x;
    const int l = threadIdx.x;
    const double* src = gram + (long)P * nchunks * (PR * PR);
    for (int e = l; e < PR * PR; e += 64) {
        double s = 0.0;
        for (int c = 0; c < nchunks; ++c) s += src[(long)c * PR * PR + e];
        G[e / PR][e % PR] = s;
        Q[e / PR][e % PR] = (e / PR == e % PR) ? 1.0 : 0.0;
    }
    if (l == 0) any_rot = 0;
    __syncthreads();
    // symmetrise (the two triangles come from different MFMA tiles)
    for (int e = l; e < PR * PR; e += 64) {
        const int i = e / PR, j = e % PR;
        if (i < j) {
            const double v = 0.5 * (G[i][j] + G[j][i]);
            G[i][j] = v;
            G[j][i] = v;
        }
    }
    __syncthreads();
    // relative off-diagonal measure before rotating
    double off = 0.0;
    for (int e = l; e < PR * PR; e += 64) {
        const int i = e / PR, j = e % PR;
        if (i < j) {
            const double dd = G[i][i] * G[j][j];
            if (dd > 0.0) off = fmax(off, fabs(G[i][j]) / sqrt(dd));
        }
    }
    for (int o = 32; o > 0; o >>= 1) off = fmax(off, __shfl_xor(off, o, 64));
    if (l == 0) atomic_max_pos(sweep_off, off);
    if (off <= tol) {
        if (l == 0) rotated[P] = 0;
        return;
    }
    for (int sw = 0; sw < inner_sweeps; ++sw) {
        int swept = 0;
        for (int rr = 0; rr < PR - 1; ++rr) {
            if (l < PR / 2) {
                const int a0 = l == 0 ? 0 : ((l - 1 + rr) % (PR - 1)) + 1;
                const int b0 = ((PR - 1 - l - 1 + rr) % (PR - 1)) + 1;
                const int a = a0 < b0 ? a0 : b0, b = a0 < b0 ? b0 : a0;
                const double gaa = G[a][a], gbb = G[b][b], gab = G[a][b];
                double c = 1.0, s = 0.0;
                if (gab != 0.0 && fabs(gab) > 1e-300 + 0.25 * tol * sqrt(fmax(gaa * gbb, 0.0))) {
                    const double tau = (gbb - gaa) / (2.0 * gab);
                    double tt;
                    if (fabs(tau) > 1e150) tt = 0.5 / tau;
                    else tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                    c = 1.0 / sqrt(1.0 + tt * tt);
                    s = tt * c;
                    swept = 1;
                }
                cs[l] = c;
                sn[l] = s;
                pa[l] = a;
                pb[l] = b;
            }
            swept = __any(swept) ? 1 : 0;
            __syncthreads();
            // rows: G <- J^T G
            for (int e = l; e < (PR / 2) * PR; e += 64) {
                const int k = e / PR, j = e % PR;
                const double c = cs[k], s = sn[k];
                if (s != 0.0) {
                    const double gp = G[pa[k]][j], gq = G[pb[k]][j];
                    G[pa[k]][j] = c * gp - s * gq;
                    G[pb[k]][j] = s * gp + c * gq;
                }
            }
            __syncthreads();
            // columns: G <- G J, Q <- Q J
            for (int e = l; e < (PR / 2) * PR; e += 64) {
                const int k = e / PR, i = e % PR;
                const double c = cs[k], s = sn[k];
                if (s != 0.0) {
                    const double gp = G[i][pa[k]], gq = G[i][pb[k]];
                    G[i][pa[k]] = c * gp - s * gq;
                    G[i][pb[k]] = s * gp + c * gq;
                    const double qp = Q[i][pa[k]], qq = Q[i][pb[k]];
                    Q[i][pa[k]] = c * qp - s * qq;
                    Q[i][pb[k]] = s * qp + c * qq;
                }
            }
            __syncthreads();
            if (swept && l == 0) any_rot = 1;
        }
        __syncthreads();
        if (!__any(swept)) break;
    }
    __syncthreads();
    // One Newton-Schulz step towards the nearest orthogonal matrix,
    // Q <- Q (3 I - Q^T Q) / 2: the product of Givens rotations is orthogonal
    // only to a few hundred ulps, and every row meets such a rotation in each
    // round of every sweep, so the defect would otherwise accumulate.
    __shared__ double T[PR][PR + 1];
    for (int e = l; e < PR * PR; e += 64) {
        const int i = e / PR, j = e % PR;
        double acc = 0.0;
        for (int k = 0; k < PR; ++k) acc += Q[k][i] * Q[k][j];
        G[i][j] = acc;
    }
    __syncthreads();
    for (int e = l; e < PR * PR; e += 64) {
        const int i = e / PR, j = e % PR;
        double acc = 0.0;
        for (int k = 0; k < PR; ++k) acc += Q[i][k] * G[k][j];
        T[i][j] = 1.5 * Q[i][j] - 0.5 * acc;
    }
    __syncthreads();
    double* out = rot + (long)P * PR * PR;
    for (int e = l; e < PR * PR; e += 64) out[e] = T[e / PR][e % PR];
    if (l == 0) rotated[P] = any_rot;
}

__global__ __launch_bounds__(RW) void rotate_kernel(double* __restrict__ Z, int p, int ld, int r,
                                                    int nb, const double* __restrict__ rot,
                                                    const int* __restrict__ rotated) {
    const int P = blockIdx.y;
    if (!rotated[P]) return;
    __shared__ double Q[PR * PR];
    const double* src = rot + (long)P * PR * PR;
    for (int e = threadIdx.x; e < PR * PR; e += RW) Q[e] = src[e];
    __syncthreads();
    const int c = blockIdx.x * RW + threadIdx.x;
    if (c >= ld) return;
    double x[PR];
    long off[PR];
#pragma unroll
    for (int lr = 0; lr < PR; ++lr) {
        const int row = pair_row(P, lr, r, nb);
        off[lr] = row < p ? (long)row * ld + c : -1;
        x[lr] = off[lr] >= 0 ? Z[off[lr]] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < PR; ++i) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < PR; ++k) s += Q[k * PR + i] * x[k];
        if (off[i] >= 0) Z[off[i]] = s;
    }
}

__global__ __launch_bounds__(256) void row_norms_kernel(const double* __restrict__ Z, int q, int ld,
                                                        double* __restrict__ norms) {
    __shared__ double sh[4];
    const int i = blockIdx.x;
    double acc = 0.0;
    for (int c = threadIdx.x; c < q; c += 256) {
        const double v = Z[(long)i * ld + c];
        acc += v * v;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) norms[i] = sqrt(sh[0] + sh[1] + sh[2] + sh[3]);
}

__global__ void gather_rows_kernel(const double* __restrict__ Z, int ld, const int* __restrict__ perm,
                                   int k, int roff, int nr, double* __restrict__ dst) {
    const int t = blockIdx.y;
    const int r = perm[t];
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < nr; c += gridDim.x * blockDim.x)
        dst[(long)t * nr + c] = Z[(long)r * ld + roff + c];
}

// coldst[i][t] = Z[perm[t]][coff + i] through a 32 x 32 tile
__global__ void gather_cols_kernel(const double* __restrict__ Z, int ld, const int* __restrict__ perm,
                                   int k, int coff, int nc, double* __restrict__ dst) {
    __shared__ double tile[32][33];
    const int i0 = blockIdx.x * 32, t0 = blockIdx.y * 32;
    for (int yy = threadIdx.y; yy < 32; yy += blockDim.y) {
        const int t = t0 + yy, i = i0 + threadIdx.x;
        tile[yy][threadIdx.x] = (t < k && i < nc) ? Z[(long)perm[t] * ld + coff + i] : 0.0;
    }
    __syncthreads();
    for (int yy = threadIdx.y; yy < 32; yy += blockDim.y) {
        const int i = i0 + yy, t = t0 + threadIdx.x;
        if (i < nc && t < k) dst[(long)i * k + t] = tile[threadIdx.x][yy];
    }
}

// Z[i][c] = X[i][c] for c < q and the identity in columns q..q+p, where X is
// theta (dir 0, p = m rows) or theta^T (dir 1, p = n rows) for theta m x n.
__global__ void jacobi_input_kernel(const double* __restrict__ theta, int m, int n, int dir,
                                    double* __restrict__ Z, int p, int q, int ld) {
    const long total = (long)p * ld;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
        const int i = (int)(e / ld), c = (int)(e % ld);
        double v;
        if (c < q) v = dir == 0 ? theta[(long)i * n + c] : theta[(long)c * n + i];
        else v = (c - q == i) ? 1.0 : 0.0;
        Z[e] = v;
    }
}

}  // namespace

void jacobi_input(const double* theta, int m, int n, int dir, double* Z, hipStream_t s) {
    const int p = dir == 0 ? m : n, q = dir == 0 ? n : m, ld = p + q;
    const long total = (long)p * ld;
    int blocks = (int)std::min<long>(8192, (total + 255) / 256);
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(jacobi_input_kernel, dim3(blocks), dim3(256), 0, s, theta, m, n, dir, Z, p, q, ld);
    HIP_CHECK(hipGetLastError());
}

JacobiResult jacobi_rows(double* Z, int p, int q, int ld, double tol, int max_sweeps,
                         double* gram_ws, double* rot_ws, double* off_ws, double* host_off,
                         hipStream_t s) {
    JacobiResult res;
    if (p <= 1) return res;
    int nb = (p + RB - 1) / RB;
    if (nb < 2) nb = 2;
    if (nb & 1) ++nb;
    const int npairs = nb / 2;
    const int nchunks = std::max(1, (q + GW - 1) / GW);
    const int nrot = (ld + RW - 1) / RW;
    int* rotated = reinterpret_cast<int*>(off_ws + 1);
    double prev = 1e300;
    for (int sw = 0; sw < max_sweeps; ++sw) {
        fill(off_ws, 0.0, 1, s);
        for (int r = 0; r < nb - 1; ++r) {
            hipLaunchKernelGGL(gram_kernel, dim3(nchunks, npairs), dim3(256), 0, s, Z, p, q, ld, r, nb,
                               nchunks, gram_ws);
            hipLaunchKernelGGL(inner_kernel, dim3(npairs), dim3(64), 0, s, gram_ws, nchunks, p, r, nb, tol,
                               8, rot_ws, rotated, off_ws);
            hipLaunchKernelGGL(rotate_kernel, dim3(nrot, npairs), dim3(RW), 0, s, Z, p, ld, r, nb, rot_ws,
                               rotated);
        }
        HIP_CHECK(hipGetLastError());
        HIP_CHECK(hipMemcpyAsync(host_off, off_ws, sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        res.sweeps = sw + 1;
        res.last_off = *host_off;
        if (*host_off <= tol) break;
        // stagnation at the rounding floor: stop once the measure no longer drops
        if (sw >= 3 && *host_off > 0.5 * prev && *host_off < 1e3 * tol) break;
        prev = *host_off;
    }
    return res;
}

void row_norms(const double* Z, int p, int q, int ld, double* norms, hipStream_t s) {
    if (p <= 0) return;
    hipLaunchKernelGGL(row_norms_kernel, dim3(p), dim3(256), 0, s, Z, q, ld, norms);
    HIP_CHECK(hipGetLastError());
}

void gather_split(const double* Z, int ld, const int* perm, int k, int roff, int nr, double* rowdst,
                  int coff, int nc, double* coldst, hipStream_t s) {
    if (k <= 0) return;
    if (nr > 0) {
        dim3 grid(std::min(64, (nr + 255) / 256), k);
        hipLaunchKernelGGL(gather_rows_kernel, grid, dim3(256), 0, s, Z, ld, perm, k, roff, nr, rowdst);
    }
    if (nc > 0) {
        dim3 grid((nc + 31) / 32, (k + 31) / 32);
        hipLaunchKernelGGL(gather_cols_kernel, grid, dim3(32, 8), 0, s, Z, ld, perm, k, coff, nc, coldst);
    }
    HIP_CHECK(hipGetLastError());
}

}  // namespace ite
