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
// Rows are grouped in blocks of RB (16, or 32 for large p); a round-robin
// (circle) schedule pairs the blocks so that every pair meets once per sweep.
// For each pair of blocks (PR = 2 RB rows):
//   1. gram:   G = X_pair X_pair^T, summed over column chunks with FP64 MFMA;
//   2. inner:  one cyclic sweep of two-sided Jacobi rotations on the PR x PR
//              matrix in LDS; Q accumulates the rotations;
//   3. rotate: Z_pair <- Q^T Z_pair over all ld columns (FP64 MFMA).
// Pairs whose rows are already orthogonal to the working tolerance produce no
// rotation and skip step 3.  A sweep ends with one host read of the largest
// off-diagonal measure seen in it.  Larger blocks halve the number of rounds
// per sweep, and with it the traffic over the whole work matrix, at the price
// of a longer inner sweep.
#include "internal.h"

#include <algorithm>
#include <cmath>

namespace ite {
namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));

constexpr int RCOLS = 128;   // columns per rotate block

template <int RB> struct Blk {
    static constexpr int PR = 2 * RB;              // rows per pair
    static constexpr int NT = PR * PR / 16;        // inner threads: 16 entries each
    static constexpr int XS = NT / PR;             // row stride of a thread's entries
    static constexpr int GW = RB == 16 ? 256 : 128;   // columns per gram chunk
};

// Block index at position `pos` of the circle schedule in round r
// (nb blocks, nb even; position 0 is fixed).
__device__ inline int circle_block(int pos, int r, int nb) {
    return pos == 0 ? 0 : ((pos - 1 + r) % (nb - 1)) + 1;
}

// Local row lr of pair P in round r; the first RB local rows always belong to
// the block with the lower index, so that the sorting rotations below move
// larger rows towards lower global indices.
template <int RB>
__device__ inline int pair_row(int P, int lr, int r, int nb) {
    const int b0 = circle_block(P, r, nb);
    const int b1 = circle_block(nb - 1 - P, r, nb);
    const int bi = b0 < b1 ? b0 : b1, bj = b0 < b1 ? b1 : b0;
    return lr < RB ? bi * RB + lr : bj * RB + (lr - RB);
}

template <int RB>
__global__ __launch_bounds__(256) void gram_kernel(const double* __restrict__ Z, int p, int q, int ld, int r,
                                                   int nb, int nchunks, double* __restrict__ gram) {
    constexpr int PR = Blk<RB>::PR, GW = Blk<RB>::GW;
    __shared__ double Xs[PR][GW + 1];
    const int P = blockIdx.y, chunk = blockIdx.x;
    const int c0 = chunk * GW;
    const int t = threadIdx.x;
    for (int e = t; e < PR * GW; e += 256) {
        const int lr = e / GW, cc = e % GW;
        const int c = c0 + cc;
        const int row = pair_row<RB>(P, lr, r, nb);
        Xs[lr][cc] = (row < p && c < q) ? Z[(long)row * ld + c] : 0.0;
    }
    __syncthreads();
    const int lane = t & 63, w = t >> 6;
    const int l16 = lane & 15, kg = lane >> 4;
    constexpr int NTL = PR / 16;                  // tiles per side
    double* out = gram + ((long)P * nchunks + chunk) * (PR * PR);
    for (int tile = w; tile < NTL * NTL; tile += 4) {
        const int I = tile / NTL, J = tile % NTL;
        d4_t acc = {0, 0, 0, 0};
        for (int k0 = 0; k0 < GW; k0 += 4)
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Xs[I * 16 + l16][k0 + kg], Xs[J * 16 + l16][k0 + kg],
                                                       acc, 0, 0, 0);
        // FP64 MFMA accumulator element rr of lane group kg is tile row 4 rr + kg
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) out[(I * 16 + 4 * rr + kg) * PR + J * 16 + l16] = acc[rr];
    }
}

__device__ inline void atomic_max_pos(double* addr, double v) {
    // non-negative doubles order like their bit patterns
    atomicMax(reinterpret_cast<unsigned long long*>(addr), (unsigned long long)__double_as_longlong(v));
}

// Orthogonality measure of rows i, j with Gram entries g_ii, g_jj, g_ij:
//   |g_ij| / (d_i d_j + kappa s1 (d_i + d_j)),   d = sqrt(g), s1 ~ sigma_max.
// The second term is the rounding floor: rotations with large rows leave an
// absolute error of order eps s1 in every row, so small rows cannot be made
// orthogonal relative to their own length (their singular values and
// vectors are then accurate in absolute terms, as for any backward-stable
// SVD).
__device__ inline double off_den(double gi, double gj, double kappa_s1) {
    const double di = sqrt(fmax(gi, 0.0)), dj = sqrt(fmax(gj, 0.0));
    return di * dj + kappa_s1 * (di + dj);
}

// One workgroup per pair: sum the chunk partials, then one cyclic sweep of
// two-sided Jacobi rotations on the PR x PR Gram matrix (each rotation the
// one of the two diagonalising angles that keeps the larger row at the lower
// index), then a Newton-Schulz step on the accumulated Q; writes Q and
// whether any rotation was applied.  sigma1sq: largest row norm squared seen
// in the previous sweep (0: use this pair's own).
//
// The PR/2 disjoint rotations of a round act as new_i = al_i old_i + be_i
// old_partner(i) on rows and columns, so every entry of G' = J^T G J and of
// Q' = Q J is an independent combination of at most four old entries: one
// double-buffered update per round with all LDS loads of a thread in flight
// together.  Thread t owns column t % PR and rows t / PR + XS u, u < 16.
template <int RB>
__global__ __launch_bounds__(Blk<RB>::NT) void inner_kernel(const double* __restrict__ gram, int nchunks, int p,
                                                            int r, int nb, double tol, double kappa,
                                                            double sigma1sq, double* __restrict__ rot,
                                                            int* __restrict__ rotated,
                                                            double* __restrict__ sweep_off) {
    constexpr int PR = Blk<RB>::PR, NT = Blk<RB>::NT, XS = Blk<RB>::XS;
    __shared__ double Gb[2][PR][PR + 1];
    __shared__ double Qb[2][PR][PR + 1];
    __shared__ double al[PR], be[PR];
    __shared__ int part[PR];
    __shared__ double red[NT / 64];
    // one slot per round parity: a wave that skips a round without rotations
    // must not overwrite the flag another wave is still reading
    __shared__ int flag[2];
    const int P = blockIdx.x;
    const int t = threadIdx.x;
    const int y = t % PR, xh = t / PR;
    const double* src = gram + (long)P * nchunks * (PR * PR);
    {
        // chunk-outer so that the 16 loads of a chunk are in flight together
        double s[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) s[u] = 0.0;
        for (int c = 0; c < nchunks; ++c) {
            const double* g = src + (long)c * PR * PR + y;
            double v[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) v[u] = g[(xh + XS * u) * PR];
#pragma unroll
            for (int u = 0; u < 16; ++u) s[u] += v[u];
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int x = xh + XS * u;
            Gb[0][x][y] = s[u];
            Qb[0][x][y] = (x == y) ? 1.0 : 0.0;
        }
    }
    __syncthreads();
    // symmetrise (the two triangles come from different MFMA tiles)
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int x = xh + XS * u;
        if (x < y) {
            const double v = 0.5 * (Gb[0][x][y] + Gb[0][y][x]);
            Gb[0][x][y] = v;
            Gb[0][y][x] = v;
        }
    }
    __syncthreads();
    // off-diagonal measure before rotating; largest diagonal for the next sweep
    double gmax_local = 0.0;
    for (int i = 0; i < PR; ++i) gmax_local = fmax(gmax_local, Gb[0][i][i]);
    const double kappa_s1 = kappa * sqrt(fmax(sigma1sq, gmax_local));
    double off = 0.0;
    {
        const double gyy = Gb[0][y][y];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int x = xh + XS * u;
            if (x < y) {
                const double den = off_den(Gb[0][x][x], gyy, kappa_s1);
                if (den > 0.0) off = fmax(off, fabs(Gb[0][x][y]) / den);
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) off = fmax(off, __shfl_xor(off, o, 64));
    if ((t & 63) == 0) red[t >> 6] = off;
    __syncthreads();
    off = red[0];
    for (int i = 1; i < NT / 64; ++i) off = fmax(off, red[i]);
    if (t == 0) {
        atomic_max_pos(sweep_off, off);
        atomic_max_pos(sweep_off + 1, gmax_local);
    }
    if (off <= tol) {
        if (t == 0) rotated[P] = 0;
        return;
    }
    int cur = 0;
    bool swept = false;
    for (int rr = 0; rr < PR - 1; ++rr) {
        if (t < 64) {
            bool mine = false;
            if (t < PR / 2) {
                const int a0 = t == 0 ? 0 : ((t - 1 + rr) % (PR - 1)) + 1;
                const int b0 = ((PR - 1 - t - 1 + rr) % (PR - 1)) + 1;
                const int a = a0 < b0 ? a0 : b0, b = a0 < b0 ? b0 : a0;
                const double gaa = Gb[cur][a][a], gbb = Gb[cur][b][b], gab = Gb[cur][a][b];
                double c = 1.0, s = 0.0;
                if (gab != 0.0 && fabs(gab) > 0.25 * tol * off_den(gaa, gbb, kappa_s1)) {
                    const double tau = (gbb - gaa) / (2.0 * gab);
                    double tt;
                    if (fabs(tau) > 1e150) tt = 0.5 / tau;
                    else tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                    c = 1.0 / sqrt(1.0 + tt * tt);
                    s = tt * c;
                    // the other diagonalising angle if this one leaves the
                    // smaller row at the lower index
                    const double naa = c * c * gaa - 2.0 * c * s * gab + s * s * gbb;
                    const double nbb = s * s * gaa + 2.0 * c * s * gab + c * c * gbb;
                    if (naa < nbb) {
                        const double c0 = c;
                        c = -s;
                        s = c0;
                    }
                    mine = true;
                }
                // new_a = c a - s b, new_b = s a + c b
                al[a] = c;
                be[a] = -s;
                al[b] = c;
                be[b] = s;
                part[a] = b;
                part[b] = a;
            }
            const bool any = __any(mine);
            if (t == 0) flag[rr & 1] = any ? 1 : 0;
        }
        __syncthreads();
        if (!flag[rr & 1]) continue;   // uniform: every thread reads the flag after the barrier
        swept = true;
        const int nxt = cur ^ 1;
        const int yp = part[y];
        const double ay = al[y], by = be[y];
        double gv[16], qv[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int x = xh + XS * u;
            const int xp = part[x];
            const double ax = al[x], bx = be[x];
            gv[u] = ax * (ay * Gb[cur][x][y] + by * Gb[cur][x][yp]) + bx * (ay * Gb[cur][xp][y] + by * Gb[cur][xp][yp]);
            qv[u] = ay * Qb[cur][x][y] + by * Qb[cur][x][yp];
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int x = xh + XS * u;
            Gb[nxt][x][y] = gv[u];
            Qb[nxt][x][y] = qv[u];
        }
        __syncthreads();
        cur = nxt;
    }
    // One Newton-Schulz step towards the nearest orthogonal matrix,
    // Q <- Q (3 I - Q^T Q) / 2: the product of Givens rotations is orthogonal
    // only to a few hundred ulps, and every row meets such a rotation in each
    // round of every sweep, so the defect would otherwise accumulate.
    double (*Q)[PR + 1] = Qb[cur];
    double (*S)[PR + 1] = Gb[cur];
    double (*T)[PR + 1] = Gb[cur ^ 1];
    {
        double acc[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) acc[u] = 0.0;
        for (int k = 0; k < PR; ++k) {
            const double qky = Q[k][y];
#pragma unroll
            for (int u = 0; u < 16; ++u) acc[u] += Q[k][xh + XS * u] * qky;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 16; ++u) S[xh + XS * u][y] = acc[u];
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 16; ++u) acc[u] = 0.0;
        for (int k = 0; k < PR; ++k) {
            const double sky = S[k][y];
#pragma unroll
            for (int u = 0; u < 16; ++u) acc[u] += Q[xh + XS * u][k] * sky;
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int x = xh + XS * u;
            T[x][y] = 1.5 * Q[x][y] - 0.5 * acc[u];
        }
    }
    __syncthreads();
    double* out = rot + (long)P * PR * PR;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int x = xh + XS * u;
        out[x * PR + y] = T[x][y];
    }
    if (t == 0) rotated[P] = swept ? 1 : 0;
}

// Z_pair <- Q^T Z_pair on a chunk of RCOLS columns with FP64 MFMA: the pair's
// rows of the chunk and Q are staged in LDS; the (PR/16) x (RCOLS/16) output
// tiles are dealt round-robin to the four wavefronts.
template <int RB>
__global__ __launch_bounds__(256) void rotate_kernel(double* __restrict__ Z, int p, int ld, int r, int nb,
                                                     const double* __restrict__ rot,
                                                     const int* __restrict__ rotated) {
    constexpr int PR = Blk<RB>::PR;
    constexpr int NTR = PR / 16, NTC = RCOLS / 16, TPW = NTR * NTC / 4;
    const int P = blockIdx.y;
    if (!rotated[P]) return;
    __shared__ double Qs[PR][PR + 1];        // Q[k][m]
    __shared__ double Zs[PR][RCOLS + 1];     // pair rows of the chunk
    const double* src = rot + (long)P * PR * PR;
    const int t = threadIdx.x;
    for (int e = t; e < PR * PR; e += 256) Qs[e / PR][e % PR] = src[e];
    const int c0 = blockIdx.x * RCOLS;
    for (int e = t; e < PR * RCOLS; e += 256) {
        const int lr = e / RCOLS, cc = e % RCOLS;
        const int c = c0 + cc;
        const int row = pair_row<RB>(P, lr, r, nb);
        Zs[lr][cc] = (row < p && c < ld) ? Z[(long)row * ld + c] : 0.0;
    }
    __syncthreads();
    const int lane = t & 63, w = t >> 6;
    const int l16 = lane & 15, kg = lane >> 4;
    d4_t acc[TPW];
#pragma unroll
    for (int i = 0; i < TPW; ++i) acc[i] = d4_t{0, 0, 0, 0};
#pragma unroll
    for (int k0 = 0; k0 < PR; k0 += 4) {
        const int k = k0 + kg;
#pragma unroll
        for (int i = 0; i < TPW; ++i) {
            const int tile = w + 4 * i;
            const int tm = tile % NTR, tn = tile / NTR;
            acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(Qs[k][tm * 16 + l16], Zs[k][tn * 16 + l16], acc[i], 0, 0,
                                                          0);
        }
    }
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
        const int tile = w + 4 * i;
        const int tm = tile % NTR, tn = tile / NTR;
        const int c = c0 + tn * 16 + l16;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const int m = tm * 16 + 4 * rr + kg;      // FP64 MFMA accumulator row
            const int row = pair_row<RB>(P, m, r, nb);
            if (row < p && c < ld) Z[(long)row * ld + c] = acc[i][rr];
        }
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

namespace {

// Rows per block: 16 for small matrices, 32 from p = 256 on (fewer rounds).
inline int block_rows(int p) { return p >= 256 ? 32 : 16; }

template <int RB>
void ws_sizes(int p, int q, size_t* gram, size_t* rot, size_t* off) {
    constexpr int PR = Blk<RB>::PR, GW = Blk<RB>::GW;
    int nb = (p + RB - 1) / RB;
    if (nb < 2) nb = 2;
    if (nb & 1) ++nb;
    const size_t npairs = nb / 2, nchunks = std::max(1, (q + GW - 1) / GW);
    *gram = npairs * nchunks * PR * PR;
    *rot = npairs * PR * PR;
    *off = npairs + 16;
}

template <int RB>
JacobiResult run_jacobi(double* Z, int p, int q, int ld, double tol, int max_sweeps, double* gram_ws,
                        double* rot_ws, double* off_ws, double* host_off, hipStream_t s) {
    constexpr int GW = Blk<RB>::GW, NT = Blk<RB>::NT;
    JacobiResult res;
    int nb = (p + RB - 1) / RB;
    if (nb < 2) nb = 2;
    if (nb & 1) ++nb;
    const int npairs = nb / 2;
    const int nchunks = std::max(1, (q + GW - 1) / GW);
    const int nrot = (ld + RCOLS - 1) / RCOLS;
    // off_ws[0]: largest off-diagonal measure of the sweep, off_ws[1]: largest
    // row norm squared seen in it, then one int per pair (rotated flag)
    int* rotated = reinterpret_cast<int*>(off_ws + 2);
    constexpr double kappa = 1e-3;
    double prev = 1e300, sigma1sq = 0.0;
    for (int sw = 0; sw < max_sweeps; ++sw) {
        fill(off_ws, 0.0, 2, s);
        for (int r = 0; r < nb - 1; ++r) {
            hipLaunchKernelGGL((gram_kernel<RB>), dim3(nchunks, npairs), dim3(256), 0, s, Z, p, q, ld, r, nb,
                               nchunks, gram_ws);
            hipLaunchKernelGGL((inner_kernel<RB>), dim3(npairs), dim3(NT), 0, s, gram_ws, nchunks, p, r, nb, tol,
                               kappa, sigma1sq, rot_ws, rotated, off_ws);
            hipLaunchKernelGGL((rotate_kernel<RB>), dim3(nrot, npairs), dim3(256), 0, s, Z, p, ld, r, nb, rot_ws,
                               rotated);
        }
        HIP_CHECK(hipGetLastError());
        HIP_CHECK(hipMemcpyAsync(host_off, off_ws, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        sigma1sq = host_off[1];
        res.sweeps = sw + 1;
        res.last_off = *host_off;
        if (*host_off <= tol) break;
        // stagnation at the rounding floor: stop once the measure no longer drops
        if (sw >= 3 && *host_off > 0.5 * prev && *host_off < 1e3 * tol) break;
        prev = *host_off;
    }
    return res;
}

}  // namespace

void jacobi_workspace(int p, int q, size_t* gram, size_t* rot, size_t* off) {
    if (block_rows(p) == 32) ws_sizes<32>(p, q, gram, rot, off);
    else ws_sizes<16>(p, q, gram, rot, off);
}

JacobiResult jacobi_rows(double* Z, int p, int q, int ld, double tol, int max_sweeps, double* gram_ws,
                         double* rot_ws, double* off_ws, double* host_off, hipStream_t s) {
    if (p <= 1) return JacobiResult{};
    if (block_rows(p) == 32) return run_jacobi<32>(Z, p, q, ld, tol, max_sweeps, gram_ws, rot_ws, off_ws, host_off, s);
    return run_jacobi<16>(Z, p, q, ld, tol, max_sweeps, gram_ws, rot_ws, off_ws, host_off, s);
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
