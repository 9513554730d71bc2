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
// Up to 64 rows one workgroup runs the whole Jacobi (blocks of 16 rows up to
// 32 rows, of 32 up to 64).  Beyond that the rows are grouped in blocks of
// RB = 32; a round-robin (circle) schedule pairs the blocks so that every
// pair meets once per sweep.
// For each pair of blocks (PR = 2 RB rows):
//   1. gram:   G = X_pair X_pair^T, summed over column chunks with FP64 MFMA;
//   2. inner:  one cyclic sweep of two-sided Jacobi rotations on the PR x PR
//              matrix in LDS (in FP32 while the previous sweep's measure is
//              above 1e-3, the measure itself always FP64); Q accumulates
//              the rotations and is made orthogonal to FP64 rounding by
//              Newton-Schulz steps;
//   3. rotate: Z_pair <- Q^T Z_pair over all ld columns (FP64 MFMA).
// Step 3 of a round and step 1 of the next are one launch
// (the data columns alternate between Z and a second buffer), and the
// identity part of step 3 runs inside the next round's inner launch.  Pairs
// whose rows are already orthogonal to the working tolerance produce no
// rotation.  A sweep ends with one host read of the largest off-diagonal
// measure seen in it; in the quadratic phase one product X X^T checks all row
// pairs at once instead of a sweep that would only confirm convergence.
// Larger blocks halve the number of rounds per sweep, and with it the traffic
// over the whole work matrix, at the price of a longer inner sweep.
#include "internal.h"
#include "wave.h"

#include <algorithm>
#include <cmath>
#include <type_traits>

namespace ite {
namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

template <int RB> struct Blk {
    static constexpr int PR = 2 * RB;              // rows per pair
    static constexpr int NT = PR * PR / 8;         // inner threads: 8 entries of a PR x PR matrix each
    static constexpr int XS = NT / PR;             // row stride of a thread's entries
    static constexpr int NTI = NT + 64;            // inner kernel: NT update threads + one angle wavefront
    static constexpr int GW = RB == 16 ? 256 : 128;   // columns per LDS stage of the gram kernel
    static constexpr int GS = 2;                   // stages per gram chunk
    static constexpr int GC = GW * GS;             // columns per gram chunk
    static constexpr int UW = 16 * (NT / 64) * 4;  // identity-part columns per rotating inner workgroup
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

// 4 GRAM_KS wavefronts: wavefront w forms tiles (w mod 4), (w mod 4) + 4, ...
// over the part w / 4 of each stage's columns; the parts are summed in LDS.
constexpr int GRAM_KS = 2, GRAM_NT = 256 * GRAM_KS;
template <int RB>
__global__ __launch_bounds__(GRAM_NT) void gram_kernel(const double* __restrict__ Z, int p, int q, int ld, int r,
                                                       int nb, int nchunks, double* __restrict__ gram,
                                                       unsigned long long* __restrict__ work) {
    constexpr int PR = Blk<RB>::PR, GW = Blk<RB>::GW, GS = Blk<RB>::GS;
    constexpr int NTL = PR / 16, NTILE = NTL * (NTL + 1) / 2, TPW = (NTILE + 3) / 4;
    constexpr int RPP = GRAM_NT / GW, NPASS = PR / RPP, KH = GW / GRAM_KS;
    static_assert(NPASS * RPP == PR && (GRAM_KS - 1) * 4 * TPW * 256 <= PR * (GW + 1), "gram layout");
    __shared__ double Xs[PR][GW + 1];
    const int P = blockIdx.y, chunk = blockIdx.x;
    const int t = threadIdx.x;
    const int cc = t % GW, lr0 = t / GW;
    long ro[NPASS];
#pragma unroll
    for (int u = 0; u < NPASS; ++u) {
        const int row = pair_row<RB>(P, lr0 + RPP * u, r, nb);
        ro[u] = row < p ? (long)row * ld : -1;
    }
    // all PR * GW / GRAM_NT loads of a stage in flight together; the next
    // stage is fetched while the matrix cores work on the current one
    double v[NPASS];
    {
        const int c = chunk * Blk<RB>::GC + cc;
#pragma unroll
        for (int u = 0; u < NPASS; ++u) v[u] = (ro[u] >= 0 && c < q) ? Z[ro[u] + c] : 0.0;
    }
    if (t == 0) atomicAdd(work, 1ull);
    const int lane = t & 63, w = t >> 6, wt = w & 3, kh = w >> 2;
    const int l16 = lane & 15, kg = lane >> 4;
    // the Gram is symmetric: only the tiles I <= J are formed and stored
    int ti[TPW], tj[TPW];
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
        int I = 0, J = wt + 4 * i;
        while (J >= NTL - I && I < NTL) {
            J -= NTL - I;
            ++I;
        }
        ti[i] = I;
        tj[i] = J + I;
    }
    d4_t acc[TPW];
#pragma unroll
    for (int i = 0; i < TPW; ++i) acc[i] = d4_t{0, 0, 0, 0};
    for (int st = 0; st < GS; ++st) {
        if (st > 0) __syncthreads();
#pragma unroll
        for (int u = 0; u < NPASS; ++u) Xs[lr0 + RPP * u][cc] = v[u];
        __syncthreads();
        if (st + 1 < GS) {
            const int c = chunk * Blk<RB>::GC + (st + 1) * GW + cc;
#pragma unroll
            for (int u = 0; u < NPASS; ++u) v[u] = (ro[u] >= 0 && c < q) ? Z[ro[u] + c] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < TPW; ++i) {
            if (wt + 4 * i >= NTILE) break;
            const int I = ti[i], J = tj[i];
            for (int k0 = kh * KH; k0 < (kh + 1) * KH; k0 += 4)
                acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(Xs[I * 16 + l16][k0 + kg], Xs[J * 16 + l16][k0 + kg],
                                                              acc[i], 0, 0, 0);
        }
    }
    // column parts 1.. into LDS, summed by part 0 in a fixed order
    __syncthreads();
    double* red = &Xs[0][0];
    if (kh > 0) {
#pragma unroll
        for (int i = 0; i < TPW; ++i) {
            if (wt + 4 * i >= NTILE) break;
#pragma unroll
            for (int rr = 0; rr < 4; ++rr)
                red[((((kh - 1) * 4 + wt) * TPW + i) * 4 + rr) * 64 + lane] = acc[i][rr];
        }
    }
    __syncthreads();
    if (kh == 0) {
        double* out = gram + ((long)P * nchunks + chunk) * (PR * PR);
#pragma unroll
        for (int i = 0; i < TPW; ++i) {
            if (wt + 4 * i >= NTILE) break;
            // FP64 MFMA accumulator element rr of lane group kg is tile row 4 rr + kg
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                double sum = acc[i][rr];
                for (int k = 1; k < GRAM_KS; ++k) sum += red[((((k - 1) * 4 + wt) * TPW + i) * 4 + rr) * 64 + lane];
                out[(ti[i] * 16 + 4 * rr + kg) * PR + tj[i] * 16 + l16] = sum;
            }
        }
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

// Round-robin order inside a pair, kept in position space: in every round
// the rows at positions i and i + RB are rotated together (i < RB), then the
// rows move one step along the ring 1 -> 2 -> ... -> RB-1 -> PR-1 -> PR-2
// -> ... -> RB -> 1 (position 0 stays).  After PR - 1 rounds every two rows
// have met once and every row is back at its starting position.  Keeping
// the partners at a fixed distance makes every update a 2 x 2 block update
// with regular LDS addresses.
template <int PR>
__device__ inline int ring_next(int pos) {
    constexpr int H = PR / 2;
    if (pos == 0) return 0;
    if (pos < H - 1) return pos + 1;
    if (pos == H - 1) return PR - 1;
    if (pos == H) return 1;
    return pos - 1;
}

// Position in round k of the row that is at `pos` in round k + 1.
template <int PR>
__device__ inline int ring_prev(int pos) {
    constexpr int H = PR / 2;
    if (pos == 0) return 0;
    if (pos == 1) return H;
    if (pos < H) return pos - 1;
    if (pos == PR - 1) return H - 1;
    return pos + 1;
}

// Local row held at position `pos` in round k (0 <= k < PR - 1).
template <int PR>
__device__ inline int ring_row(int pos, int k) {
    constexpr int H = PR / 2, M = PR - 1;
    if (pos == 0) return 0;
    const int rg = pos < H ? pos - 1 : PR - 2 - (pos - H);
    int r0 = rg - k;
    if (r0 < 0) r0 += M;
    return r0 <= H - 2 ? r0 + 1 : H + (PR - 2 - r0);
}

// Jacobi angle of the pair (a, b) with Gram entries g_aa, g_bb, g_ab:
// tan(theta) = sign(x) y / (|x| + r), x = g_bb - g_aa, y = 2 g_ab,
// r = hypot(x, y); new_a = c a - s b, new_b = s a + c b.  Written without a
// division: with d = |x| + r, cos = d / sqrt(2 r d) and
// sin = sign(x) y / sqrt(2 r d) (x and y first scaled by a power of two, so
// that nothing overflows or underflows).  This rotation keeps the order of
// the two diagonal entries (b ends larger when x >= 0); of the two
// diagonalising angles the one that leaves the larger row at the lower local
// index (a_low: a has the lower index) is taken, by swapping (c, s) to
// (-s, c) when needed.  Returns whether the pair rotates.
template <typename T>
__device__ inline bool jacobi_angle(T gaa, T gbb, T gab, bool a_low, T& c, T& s) {
    c = T(1);
    s = T(0);
    if (gab == T(0)) return false;
    const T x = gbb - gaa, yy = T(2) * gab;
    int e;
    (void)frexp(fmax(fabs(x), fabs(yy)), &e);
    const T xs = ldexp(x, -e), ys = ldexp(yy, -e);
    // xs, ys are scaled so that xs^2 + ys^2 lies in [1/4, 2) and 2 r d in
    // [1/2, 8): in single precision the hardware square root and reciprocal
    // square root (no range reduction needed) are used directly
    T r, iw;
    if constexpr (std::is_same<T, float>::value) {
        r = __builtin_amdgcn_sqrtf(xs * xs + ys * ys);
        iw = __builtin_amdgcn_rsqf(T(2) * r * (fabs(xs) + r));
    } else {
        r = sqrt(xs * xs + ys * ys);
        iw = rsqrt(T(2) * r * (fabs(xs) + r));
    }
    const T d = fabs(xs) + r;
    c = d * iw;
    s = (x >= T(0) ? ys : -ys) * iw;
    if (a_low == (x >= T(0))) {
        const T c0 = c;
        c = -s;
        s = c0;
    }
    return true;
}

// (cos, sin) of a round's rotations in the sweep's precision.
template <typename T> struct CosSin;
template <> struct CosSin<double> {
    typedef double2 type;
    static __device__ type make(double c, double s) { return make_double2(c, s); }
};
template <> struct CosSin<float> {
    typedef float2 type;
    static __device__ type make(float c, float s) { return make_float2(c, s); }
};

// Entry (x, y) of G' = J G J^T for positions x, y of the current round, J the
// round's rotations ((cos, sin) by pair index): the same expressions as the
// 2 x 2 block updates of inner_kernel.
template <int RB, typename T>
__device__ inline T rotated_entry(const T (*G)[2 * RB + 1], const typename CosSin<T>::type* cs, int x, int y) {
    const bool rx = x >= RB, ry = y >= RB;
    const int i = rx ? x - RB : x, j = ry ? y - RB : y;
    const auto pi = cs[i], pj = cs[j];
    const T ci = pi.x, si = pi.y, cj = pj.x, sj = pj.y;
    const T g00 = G[i][j], g01 = G[i][j + RB], g10 = G[i + RB][j], g11 = G[i + RB][j + RB];
    const T t0 = rx ? si * g00 + ci * g10 : ci * g00 - si * g10;
    const T t1 = rx ? si * g01 + ci * g11 : ci * g01 - si * g11;
    return ry ? t0 * sj + t1 * cj : t0 * cj - t1 * sj;
}

// Z_pair <- Q^T Z_pair with FP64 MFMA on columns [cb, ce) of the pair's rows
// for the pair of round r, Q (Q[k][m]) staged in LDS.  NWV wavefronts stream
// 16-column slices of the pair's rows from memory straight into MFMA
// operands, fetching the next slice while the matrix cores work on the
// current one, and write the rotated values back (wavefronts own disjoint
// columns, so the update is in place).  Every thread of the workgroup calls
// this (it holds one barrier: Q must be complete in LDS after it); threads
// with `active` false only take part in the barrier.  PF: fetch one slice
// ahead (twice the operand registers); QREG: keep Q in registers across
// slices (otherwise Q is read from LDS for every slice).
template <int RB, int NWV, bool PF, bool QREG>
__device__ __forceinline__ void rotate_cols(double* __restrict__ Z, int p, int ld, int P, int r, int nb,
                                   const double (*Qs)[2 * RB + 1], int cb, int ce, int t, bool active) {
    constexpr int PR = 2 * RB;
    constexpr int NTM = PR / 16, KS = PR / 4, STRIDE = 16 * NWV;   // row tiles, k steps, slice stride
    const int lane = t & 63, w = t >> 6;
    const int l16 = lane & 15, kg = lane >> 4;
    // element offsets of the operand rows this lane reads and of the rows it
    // writes (-1: past the matrix; p ld < 2^31 is checked by the caller)
    int rk[KS], ro[NTM * 4];
    double b[KS], bn[PF ? KS : 1];
    const int c0 = cb + w * 16 + l16;
    if (active) {
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int row = pair_row<RB>(P, 4 * ks + kg, r, nb);
            rk[ks] = row < p ? row * ld : -1;
        }
#pragma unroll
        for (int m4 = 0; m4 < NTM * 4; ++m4) {
            const int row = pair_row<RB>(P, 4 * m4 + kg, r, nb);    // FP64 MFMA accumulator row
            ro[m4] = row < p ? row * ld : -1;
        }
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) b[ks] = (rk[ks] >= 0 && c0 < ce) ? Z[rk[ks] + c0] : 0.0;
    }
    __syncthreads();
    if (!active) return;
    const int nit = (ce - cb + STRIDE - 1) / STRIDE;
    for (int it = 0; it < nit; ++it) {
        const int c = c0 + it * STRIDE, cn = c + STRIDE;
        if (!QREG) asm volatile("" ::: "memory");   // keeps the Q operand loads inside the loop
        if (PF && it + 1 < nit) {
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) bn[PF ? ks : 0] = (rk[ks] >= 0 && cn < ce) ? Z[rk[ks] + cn] : 0.0;
        }
        if (!PF && it > 0) {
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) b[ks] = (rk[ks] >= 0 && c < ce) ? Z[rk[ks] + c] : 0.0;
        }
        d4_t acc[NTM];
#pragma unroll
        for (int tm = 0; tm < NTM; ++tm) acc[tm] = d4_t{0, 0, 0, 0};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
#pragma unroll
            for (int tm = 0; tm < NTM; ++tm)
                acc[tm] = __builtin_amdgcn_mfma_f64_16x16x4f64(Qs[4 * ks + kg][tm * 16 + l16], b[ks], acc[tm],
                                                               0, 0, 0);
#pragma unroll
        for (int tm = 0; tm < NTM; ++tm)
#pragma unroll
            for (int rr = 0; rr < 4; ++rr)
                if (ro[4 * tm + rr] >= 0 && c < ce) Z[ro[4 * tm + rr] + c] = acc[tm][rr];
        if (PF) {
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) b[ks] = bn[PF ? ks : 0];
        }
    }
}

// Shared memory of one block pair's inner sweep: the Gram (two buffers, by
// round parity), the accumulated rotation (two buffers), the angles of a
// round and of the next, reduction slots.
template <int RB> struct PairLDS {
    static constexpr int PR = 2 * RB, NW = Blk<RB>::NT / 64;
    double Gb[2][PR][PR + 1];
    __align__(16) double Ab[2][PR][PR + 2];
    double2 cs[2][RB];               // (cos, sin) of each pair's rotation, by round parity
    double red[NW], gred[NW];
    int anyrot;
};

// Buffer of PairLDS::Gb that holds Q after pair_sweep.
template <int RB> constexpr int q_buffer() { return ((2 * RB - 1) & 1) ^ 1; }

// One cyclic sweep of two-sided Jacobi rotations on the PR x PR Gram of a
// block pair (each rotation the one of the two diagonalising angles that
// keeps the larger row at the lower local index), then a Newton-Schulz step
// on the accumulated rotation.  On entry Gb[0] holds the Gram's 16 x 16
// tiles on and above the diagonal and Ab[0] the identity (written by the
// caller; this function begins with a barrier).  sigma1sq: largest row norm
// squared seen in the previous sweep (0: use this pair's own).  sweep_off
// (may be null) receives, by atomic maximum, the off-diagonal measure and the
// largest diagonal entry.  Returns 0 when the rows are already orthogonal to
// the tolerance (nothing done), else 1 + whether any rotation was applied;
// then Q (new row m = sum_k Q[k][m] old row k) is in Gb[q_buffer<RB>()].
//
// NT threads form G' = J G J^T of each round as RB x RB independent 2 x 2
// block updates (rows and columns {i, i + RB} x {j, j + RB}) and the
// accumulated rotation A' = J A as row-pair updates, both written straight to
// the next round's positions in the other LDS buffer.  A holds the new rows
// (positions) against the original local rows (columns); Q = A^T.  One more
// wavefront computes the angles one round ahead: from G and the angles of
// round k it forms the three entries of G' each pair of round k + 1 needs and
// that pair's angle, while the update of round k runs, so a round costs one
// barrier.
template <int RB, typename GT = double>
__device__ __forceinline__ int pair_sweep(PairLDS<RB>& sh, double tol, double kappa, double sigma1sq, double* sweep_off,
                          double& off_out) {
    constexpr int PR = Blk<RB>::PR, NT = Blk<RB>::NT, XS = Blk<RB>::XS, EPT = PR / XS;
    constexpr int QPT = RB * RB / NT, IS = NT / RB;     // 2 x 2 blocks per thread, their row stride
    constexpr int NW = NT / 64, NTL = PR / 16;          // update wavefronts, 16 x 16 tiles per side
    static_assert(QPT * NT == RB * RB && EPT * NT == PR * PR && (RB * PR / 2) % NT == 0, "thread layout");
    static_assert((NTL * NTL) % NW == 0, "tiles per wavefront");
    auto& Gb = sh.Gb;
    auto& Ab = sh.Ab;
    // angles in the sweep's precision, over sh.cs
    typedef typename CosSin<GT>::type CS2;
    CS2(&cs)[2][RB] = *reinterpret_cast<CS2(*)[2][RB]>(&sh.cs[0][0]);
    auto& red = sh.red;
    auto& gred = sh.gred;
    int& anyrot = sh.anyrot;
    const int t = threadIdx.x;
    const bool upd = t < NT;                      // update thread (else: the angle wavefront)
    const int al = t - NT;                        // lane of the angle wavefront
    const int y = t % PR, xh = t / PR;
    if (t == 0) anyrot = 0;
    __syncthreads();
    // symmetrise: tiles below the diagonal were not formed and take the
    // transpose; inside a diagonal tile the two triangles come from different
    // MFMA lanes and are averaged
    if (upd) {
        double dm = 0.0;
#pragma unroll
        for (int u = 0; u < EPT; ++u) {
            const int x = xh + XS * u;
            if ((x >> 4) > (y >> 4)) {
                Gb[0][x][y] = Gb[0][y][x];
            } else if ((x >> 4) == (y >> 4) && x < y) {
                const double v = 0.5 * (Gb[0][x][y] + Gb[0][y][x]);
                Gb[0][x][y] = v;
                Gb[0][y][x] = v;
            } else if (x == y) {
                dm = fmax(dm, Gb[0][x][y]);
            }
        }
        dm = wave_max_nonneg(dm);
        if ((t & 63) == 0) gred[t >> 6] = dm;
    }
    __syncthreads();
    // off-diagonal measure before rotating; largest diagonal for the next sweep
    double gmax_local = gred[0];
    for (int i = 1; i < NW; ++i) gmax_local = fmax(gmax_local, gred[i]);
    const double kappa_s1 = kappa * sqrt(fmax(sigma1sq, gmax_local));
    double off = 0.0;
    double gv[EPT];     // this thread's entries, kept for the single-precision copy
    if (upd) {
        const double gyy = Gb[0][y][y];
#pragma unroll
        for (int u = 0; u < EPT; ++u) {
            const int x = xh + XS * u;
            gv[u] = Gb[0][x][y];
            if (x < y) {
                const double den = off_den(Gb[0][x][x], gyy, kappa_s1);
                if (den > 0.0) off = fmax(off, fabs(gv[u]) / den);
            }
        }
    }
    off = wave_max_nonneg(off);
    if (upd && (t & 63) == 0) red[t >> 6] = off;
    __syncthreads();
    off = red[0];
    for (int i = 1; i < NW; ++i) off = fmax(off, red[i]);
    off_out = off;
    if (t == 0 && sweep_off) {
        atomic_max_pos(sweep_off, off);
        atomic_max_pos(sweep_off + 1, gmax_local);
    }
    if (off <= tol) return 0;
    // the sweep's copies of G, in GT: for single precision they take the
    // space of Gb[0] (two float matrices), converted after the measure above
    GT(&Gw)[2][PR][PR + 1] = *reinterpret_cast<GT(*)[2][PR][PR + 1]>(&Gb[0][0][0]);
    static_assert(sizeof(GT) == sizeof(double) || 2 * sizeof(GT) * PR * (PR + 1) <= sizeof(Gb[0]), "G fits");
    // likewise the accumulated rotation: in GT, over Ab[0] for single
    // precision (started at the identity here)
    GT(&Aw)[2][PR][PR + 2] = *reinterpret_cast<GT(*)[2][PR][PR + 2]>(&Ab[0][0][0]);
    if constexpr (!std::is_same<GT, double>::value) {
        // every read of the FP64 Gram happened before the barrier above
        if (upd) {
#pragma unroll
            for (int u = 0; u < EPT; ++u) {
                const int x = xh + XS * u;
                Gw[0][x][y] = GT(gv[u]);
                Aw[0][x][y] = x == y ? GT(1) : GT(0);
            }
        }
        __syncthreads();
    }
    // angles of round 0
    if (!upd && al < RB) {
        GT c, s;
        if (jacobi_angle<GT>(Gw[0][al][al], Gw[0][al + RB][al + RB], Gw[0][al][al + RB],
                             ring_row<PR>(al, 0) < ring_row<PR>(al + RB, 0), c, s))
            anyrot = 1;
        cs[0][al] = CosSin<GT>::make(c, s);
    }
    __syncthreads();
    // fixed per update thread: the column pair j of its 2 x 2 blocks, the
    // column l of its entries of A
    const int jq = t % RB;
    const int pj0 = ring_next<PR>(jq), pj1 = ring_next<PR>(jq + RB);
    // entries of A per thread: columns (ca, ca + 1) of rows i and i + RB for
    // JC row pairs i (16-byte LDS accesses; rows padded to an even length);
    // the next-round positions of a thread's rows are fixed, computed once
    constexpr int JC = RB * (PR / 2) / NT, JCS = NT / (PR / 2);
    const int ca = 2 * (t % (PR / 2));
    int pa0[JC], pa1[JC], pq0[QPT], pq1[QPT];
#pragma unroll
    for (int u = 0; u < JC; ++u) {
        pa0[u] = ring_next<PR>(t / (PR / 2) + JCS * u);
        pa1[u] = ring_next<PR>(t / (PR / 2) + JCS * u + RB);
    }
#pragma unroll
    for (int u = 0; u < QPT; ++u) {
        pq0[u] = ring_next<PR>(t / RB + IS * u);
        pq1[u] = ring_next<PR>(t / RB + IS * u + RB);
    }
    int cur = 0;
    for (int k = 0; k < PR - 1; ++k) {
        const int pb = k & 1, nxt = cur ^ 1;
        if (upd) {
            const CS2 pj = cs[pb][jq];
            const GT cj = pj.x, sj = pj.y;
            GT nv[QPT][4];
#pragma unroll
            for (int u = 0; u < QPT; ++u) {
                const int i = t / RB + IS * u;
                const CS2 pi = cs[pb][i];
                const GT ci = pi.x, si = pi.y;
                const GT g00 = Gw[cur][i][jq], g01 = Gw[cur][i][jq + RB];
                const GT g10 = Gw[cur][i + RB][jq], g11 = Gw[cur][i + RB][jq + RB];
                const GT t00 = ci * g00 - si * g10, t01 = ci * g01 - si * g11;
                const GT t10 = si * g00 + ci * g10, t11 = si * g01 + ci * g11;
                nv[u][0] = t00 * cj - t01 * sj;
                nv[u][1] = t00 * sj + t01 * cj;
                nv[u][2] = t10 * cj - t11 * sj;
                nv[u][3] = t10 * sj + t11 * cj;
            }
            using GT2 = typename std::conditional<std::is_same<GT, double>::value, double2, float2>::type;
            GT2 na[JC][2];
#pragma unroll
            for (int u = 0; u < JC; ++u) {
                const int i = t / (PR / 2) + JCS * u;
                const CS2 pi = cs[pb][i];
                const GT ci = pi.x, si = pi.y;
                const GT2 a0 = *reinterpret_cast<const GT2*>(&Aw[cur][i][ca]);
                const GT2 a1 = *reinterpret_cast<const GT2*>(&Aw[cur][i + RB][ca]);
                na[u][0].x = ci * a0.x - si * a1.x;
                na[u][0].y = ci * a0.y - si * a1.y;
                na[u][1].x = si * a0.x + ci * a1.x;
                na[u][1].y = si * a0.y + ci * a1.y;
            }
#pragma unroll
            for (int u = 0; u < QPT; ++u) {
                const int pi0 = pq0[u], pi1 = pq1[u];
                Gw[nxt][pi0][pj0] = nv[u][0];
                Gw[nxt][pi0][pj1] = nv[u][1];
                Gw[nxt][pi1][pj0] = nv[u][2];
                Gw[nxt][pi1][pj1] = nv[u][3];
            }
#pragma unroll
            for (int u = 0; u < JC; ++u) {
                *reinterpret_cast<GT2*>(&Aw[nxt][pa0[u]][ca]) = na[u][0];
                *reinterpret_cast<GT2*>(&Aw[nxt][pa1[u]][ca]) = na[u][1];
            }
        } else if (al < RB && k + 1 < PR - 1) {
            // pair al of round k + 1 sits at positions (al, al + RB) then,
            // i.e. at (a, b) now
            const int a = ring_prev<PR>(al), b = ring_prev<PR>(al + RB);
            const GT gaa = rotated_entry<RB, GT>(Gw[cur], cs[pb], a, a);
            const GT gbb = rotated_entry<RB, GT>(Gw[cur], cs[pb], b, b);
            const GT gab = rotated_entry<RB, GT>(Gw[cur], cs[pb], a, b);
            GT c, s;
            if (jacobi_angle<GT>(gaa, gbb, gab, ring_row<PR>(al, k + 1) < ring_row<PR>(al + RB, k + 1), c, s))
                anyrot = 1;
            cs[pb ^ 1][al] = CosSin<GT>::make(c, s);
        }
        __syncthreads();
        cur = nxt;
    }
    // Every row is back at its starting position.  Newton-Schulz steps
    // towards the nearest orthogonal matrix, A <- (3 I - A A^T) A / 2 =
    // A - E A / 2 with E = A A^T - I: the product of Givens rotations is
    // orthogonal only to a few hundred ulps (to about 1e-5 for the
    // single-precision sweep, whose rotations are FP32 pairs (cos, sin)
    // applied in FP32), and every row meets such a rotation in each round of
    // every sweep, so the defect would otherwise accumulate.  The step
    // squares the defect: one suffices from FP64, two from FP32 (held in
    // double in Ab[cur]).  A A^T is formed with FP64 MFMA (E must be exact to
    // the defect the step leaves); E A with FP32 MFMA from E and A rounded to
    // FP32: E is at most about 1e-5, so the product's error (a few 1e-7 of
    // E A) stays below the squared defect, and A - E A / 2 is formed in FP64.
    const int lane = t & 63, w = t >> 6;
    const int l16 = lane & 15, kg = lane >> 4;
    constexpr int TPW = NTL * NTL / NW;
    // E in FP32 over Gb[cur] (rows of PR + 4 floats: the operand reads of
    // a 16 x 4 block fall in distinct banks)
    constexpr int LE = PR + 4;
    static_assert(PR * LE * sizeof(float) <= sizeof(Gb[0]), "E fits");
    float (*E)[LE] = reinterpret_cast<float (*)[LE]>(&Gb[cur][0][0]);
    // A - E A / 2: transposed into Gb[cur ^ 1] (the final Q) or, for a first
    // step, into out; A is read as double whatever it is stored in.
    // A A^T is symmetric: only its tiles on and above the diagonal are
    // formed, each written to both of its places
    constexpr int NUT = NTL * (NTL + 1) / 2, UPW = (NUT + NW - 1) / NW;
    const int wu = __builtin_amdgcn_readfirstlane(w);
    auto ns_step = [&](auto A, double (*out)[PR + 2], bool last) {
        if (upd) {
#pragma unroll
            for (int i = 0; i < UPW; ++i) {
                const int tile = wu + NW * i;
                if (tile >= NUT) break;
                int tm = 0, tn = tile;
                while (tn >= NTL - tm) {
                    tn -= NTL - tm;
                    ++tm;
                }
                tn += tm;
                d4_t acc = {0, 0, 0, 0};
#pragma unroll
                for (int k0 = 0; k0 < PR; k0 += 4)
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(double(A[tm * 16 + l16][k0 + kg]),
                                                               double(A[tn * 16 + l16][k0 + kg]), acc, 0, 0, 0);
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) {
                    // FP64 MFMA: element rr of lane group kg is tile row 4 rr + kg
                    const int m = tm * 16 + 4 * rr + kg, n = tn * 16 + l16;
                    const float e = float(acc[rr] - (m == n ? 1.0 : 0.0));
                    E[m][n] = e;
                    if (tm != tn) E[n][m] = e;
                }
            }
        }
        __syncthreads();
        if (upd) {
#pragma unroll
            for (int i = 0; i < TPW; ++i) {
                const int tile = w + NW * i;
                const int tm = tile / NTL, tn = tile % NTL;
                f4_t acc = {0, 0, 0, 0};
#pragma unroll
                for (int k0 = 0; k0 < PR; k0 += 4)
                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(E[tm * 16 + l16][k0 + kg],
                                                               float(A[k0 + kg][tn * 16 + l16]), acc, 0, 0, 0);
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) {
                    // FP32 MFMA: element rr of lane group kg is tile row 4 kg + rr
                    const int m = tm * 16 + 4 * kg + rr, kk = tn * 16 + l16;
                    const double v = double(A[m][kk]) - 0.5 * double(acc[rr]);
                    if (last)
                        Gb[cur ^ 1][kk][m] = v;
                    else
                        out[m][kk] = v;
                }
            }
        }
        __syncthreads();
    };
    if constexpr (std::is_same<GT, double>::value) {
        ns_step(Ab[cur], nullptr, true);
    } else {
        // first step straight from the FP32 rotation (over Ab[0]) into Ab[cur]:
        // cur is odd after the PR - 1 rounds, so Ab[cur] does not overlap it
        static_assert(((PR - 1) & 1) == 1, "odd number of rounds");
        ns_step(Aw[cur], Ab[cur], false);
        ns_step(Ab[cur], nullptr, true);
    }
    return anyrot ? 2 : 1;
}

// One workgroup per pair: sum the chunk partials of the pair's Gram (tiles on
// and above the diagonal) and run pair_sweep; writes Q and whether any
// rotation was applied.
//
// Workgroups npairs and up rotate the identity part (columns q .. ld) of
// the rows of the previous round's pairs (round rprev, rotations rot_prev),
// UW columns each: that work is off the critical path of the sweep and
// fills the compute units the pairs leave idle.  work[1] counts the pairs
// swept, work[3] the identity-part columns rotated here.
template <int RB, typename GT>
__global__ __launch_bounds__(Blk<RB>::NTI) void inner_kernel(const double* __restrict__ gram, int nchunks, int p,
                                                             int r, int nb, double tol, double kappa,
                                                             double sigma1sq, double* __restrict__ rot,
                                                             int* __restrict__ rotated,
                                                             double* __restrict__ sweep_off,
                                                             unsigned long long* __restrict__ work,
                                                             double* __restrict__ Z, int ld, int q, int npairs,
                                                             int rprev, const double* __restrict__ rot_prev,
                                                             const int* __restrict__ rotated_prev, int nuch) {
    constexpr int PR = Blk<RB>::PR, NT = Blk<RB>::NT, XS = Blk<RB>::XS, EPT = PR / XS;
    constexpr int NW = NT / 64;
    constexpr int NTI = Blk<RB>::NTI, UW = Blk<RB>::UW;
    __shared__ PairLDS<RB> sh;
    if ((int)blockIdx.x >= npairs) {
        const int u = blockIdx.x - npairs, Pu = u / nuch, ch = u % nuch;
        if (!rotated_prev[Pu]) return;
        const int cb = q + ch * UW, ce = min(cb + UW, ld);
        if (threadIdx.x == 0) atomicAdd(work + 3, (unsigned long long)(ce - cb));
        const double* qsrc = rot_prev + (long)Pu * PR * PR;
        for (int e = threadIdx.x; e < PR * PR; e += NTI) sh.Gb[0][e / PR][e % PR] = qsrc[e];
        rotate_cols<RB, NW, false, false>(Z, p, ld, Pu, rprev, nb, sh.Gb[0], cb, ce, threadIdx.x, threadIdx.x < NT);
        return;
    }
    const int P = blockIdx.x;
    const int t = threadIdx.x;
    const bool upd = t < NT;
    const int y = t % PR, xh = t / PR;
    const double* src = gram + (long)P * nchunks * (PR * PR);
    if (upd) {
        // LB chunks per step so that LB EPT loads are in flight together
        // (the summation order is fixed: results do not depend on timing)
        constexpr int LB = 4;
        double s[EPT];
#pragma unroll
        for (int u = 0; u < EPT; ++u) s[u] = 0.0;
        int c = 0;
        for (; c + LB - 1 < nchunks; c += LB) {
            const double* g = src + (long)c * PR * PR + y;
            double v[LB][EPT];
#pragma unroll
            for (int h = 0; h < LB; ++h)
#pragma unroll
                for (int u = 0; u < EPT; ++u)
                    v[h][u] = ((xh + XS * u) >> 4) <= (y >> 4) ? g[(long)h * PR * PR + (xh + XS * u) * PR] : 0.0;
#pragma unroll
            for (int u = 0; u < EPT; ++u) {
                double t4 = 0.0;
#pragma unroll
                for (int h = 0; h < LB; h += 4) t4 += (v[h][u] + v[h + 1][u]) + (v[h + 2][u] + v[h + 3][u]);
                s[u] += t4;
            }
        }
        for (; c < nchunks; ++c) {
            const double* g = src + (long)c * PR * PR + y;
#pragma unroll
            for (int u = 0; u < EPT; ++u)
                if (((xh + XS * u) >> 4) <= (y >> 4)) s[u] += g[(xh + XS * u) * PR];
        }
#pragma unroll
        for (int u = 0; u < EPT; ++u) {
            const int x = xh + XS * u;
            sh.Gb[0][x][y] = s[u];
            sh.Ab[0][x][y] = (x == y) ? 1.0 : 0.0;
        }
    }
    double off;
    const int res = pair_sweep<RB, GT>(sh, tol, kappa, sigma1sq, sweep_off, off);
    if (res != 0 && t == 0) atomicAdd(work + 1, 1ull);
    // Q of every pair is written (the identity when the rows are already
    // orthogonal), so that the fused rotation reads it unconditionally
    if (upd) {
        const auto& T = sh.Gb[q_buffer<RB>()];
        double* out = rot + (long)P * PR * PR;
#pragma unroll
        for (int u = 0; u < EPT; ++u) {
            const int x = xh + XS * u;
            out[x * PR + y] = res == 0 ? (x == y ? 1.0 : 0.0) : T[x][y];
        }
    }
    if (t == 0) rotated[P] = res == 2;
}

// The whole one-sided Jacobi of p <= PR rows (a single block pair) in one
// workgroup, for small splits where launches and host round trips would
// dominate: per sweep the Gram of the rows over the first q columns (FP64
// MFMA straight from memory, tiles on and above the diagonal), pair_sweep,
// and the rotation of the rows over all ld columns; until the rows are
// orthogonal to the tolerance, the measure stagnates at the rounding floor
// (as in the multi-pair driver), or max_sweeps.  res[0]: the last measure,
// res[1]: the number of sweeps.
template <int RB>
__global__ __launch_bounds__(Blk<RB>::NTI) void single_pair_jacobi_kernel(double* __restrict__ Z, int p, int q,
                                                                          int ld, double tol, double kappa,
                                                                          int max_sweeps, double* __restrict__ res) {
    constexpr int PR = Blk<RB>::PR, NT = Blk<RB>::NT, NW = NT / 64;
    constexpr int NTL = PR / 16, NTILE = NTL * (NTL + 1) / 2;
    __shared__ PairLDS<RB> sh;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int l16 = lane & 15, kg = lane >> 4;
    double prev = 1e300, off = 0.0;
    int sweeps = 0;
    for (int sw = 0; sw < max_sweeps; ++sw) {
        sweeps = sw + 1;
        if (t < NT) {
            for (int tile = w; tile < NTILE; tile += NW) {
                int I = 0, J = tile;
                while (J >= NTL - I) {
                    J -= NTL - I;
                    ++I;
                }
                J += I;
                const int ra = I * 16 + l16, rb = J * 16 + l16;
                const double* za = Z + (long)ra * ld;
                const double* zb = Z + (long)rb * ld;
                d4_t acc = {0, 0, 0, 0};
                for (int k0 = 0; k0 < q; k0 += 4) {
                    const int c = k0 + kg;
                    const double a = (ra < p && c < q) ? za[c] : 0.0;
                    const double b = (rb < p && c < q) ? zb[c] : 0.0;
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
                }
                // FP64 MFMA accumulator element rr of lane group kg is tile row 4 rr + kg
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) sh.Gb[0][I * 16 + 4 * rr + kg][J * 16 + l16] = acc[rr];
            }
            for (int e = t; e < PR * PR; e += NT) sh.Ab[0][e / PR][e % PR] = (e / PR == e % PR) ? 1.0 : 0.0;
        }
        if (pair_sweep<RB>(sh, tol, kappa, 0.0, nullptr, off) == 0) break;
        rotate_cols<RB, NW, false, false>(Z, p, ld, 0, 0, 2, sh.Gb[q_buffer<RB>()], 0, ld, t, t < NT);
        // the next sweep's Gram reads the rotated rows: wait for the stores
        // and drop stale lines of the vector cache
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "agent");
        if (sw >= 3 && off > 0.5 * prev && off < 1e3 * tol) break;
        prev = off;
    }
    if (t == 0) {
        res[0] = off;
        res[1] = sweeps;
    }
}

// Position-to-pair bookkeeping of the circle schedule: the pair of round r
// that holds block b, and whether b is that pair's higher-indexed block.
__device__ inline void block_pair(int b, int r, int nb, int& P, int& side) {
    const int m = nb - 1;
    const int pos = b == 0 ? 0 : ((b - 1 - r) % m + m) % m + 1;
    P = pos < nb / 2 ? pos : nb - 1 - pos;
    const int b0 = circle_block(P, r, nb), b1 = circle_block(nb - 1 - P, r, nb);
    side = b == (b0 < b1 ? b0 : b1) ? 0 : 1;
}

// Round r's rotation of the data columns fused with round r + 1's Gram: one
// workgroup per pair P' of round r + 1 and column chunk (GC columns).  Its
// two blocks come from two different pairs of round r; for each, the block's
// new rows are formed from that pair's 2 RB old rows and the block's half of
// Q (FP64 MFMA, all operand loads of the chunk issued up front), written to
// the other data buffer (Xd: the old rows are read by two workgroups, so the
// update cannot be in place), and kept in LDS for the Gram partial of P'
// (tiles on and above the diagonal).  Pairs of round r without rotation
// carry Q = I (written by the inner launch), so their rows are copied.
// Eight wavefronts: wavefront w rotates the 16-column slab w mod 4 of half
// w / 4 of every 64-column slice.  Xs is not declared __restrict__: its loads
// must stay above the compiler barrier that keeps them in flight together.
template <int RB>
__global__ __launch_bounds__(512) void rotate_gram_kernel(const double* Xs, int lds,
                                                          double* __restrict__ Xd, int ldd, int p, int q, int r,
                                                          int nb, int nchunks, const double* __restrict__ rot,
                                                          double* __restrict__ gram,
                                                          unsigned long long* __restrict__ work) {
    constexpr int PR = Blk<RB>::PR, GC = Blk<RB>::GC, KS = PR / 4, SW = 64;   // slice width
    constexpr int NTL = PR / 16, NTILE = NTL * (NTL + 1) / 2, GTW = (NTILE + 7) / 8;
    static_assert(RB == 32, "two 16-row tiles per half");
    __shared__ double Qh[2][PR][RB + 1];     // Q[k][side RB + i] of each half's round-r pair
    __shared__ double Ys[2][PR][SW + 1];     // new rows of P' over a slice (two slices in flight)
    const int Pn = blockIdx.y, chunk = blockIdx.x;
    const int t = threadIdx.x, lane = t & 63;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6);   // wavefront-uniform: schedule arithmetic stays scalar
    const int l16 = lane & 15, kg = lane >> 4;
    const int rn = r + 1;
    const int bn0 = circle_block(Pn, rn, nb), bn1 = circle_block(nb - 1 - Pn, rn, nb);
    const int blk[2] = {bn0 < bn1 ? bn0 : bn1, bn0 < bn1 ? bn1 : bn0};
    int Ph[2], sh[2];
    block_pair(blk[0], r, nb, Ph[0], sh[0]);
    block_pair(blk[1], r, nb, Ph[1], sh[1]);
    // Q of both round-r pairs (the identity for pairs without rotation is
    // written by the inner launch), loaded before the data so that waiting
    // for it leaves the data loads in flight
    constexpr int QPT = 2 * PR * RB / 512;
    double qv[QPT];
#pragma unroll
    for (int u = 0; u < QPT; ++u) {
        const int e = t + 512 * u;
        const int h = e / (PR * RB), k = (e / RB) % PR, i = e % RB;
        qv[u] = rot[(long)Ph[h] * PR * PR + k * PR + sh[h] * RB + i];
    }
    if (t == 0) atomicAdd(work, (unsigned long long)min(GC, q - chunk * GC));
    // this wavefront: half hw, 16-column slab cs of each slice
    const int hw = w >> 2, csl = w & 3;
    int rk[KS], ro[2][4];
    {
        // local rows 0..RB-1 of the round-r pair are its lower-indexed block
        const int s0 = circle_block(Ph[hw], r, nb), s1 = circle_block(nb - 1 - Ph[hw], r, nb);
        const int bi = s0 < s1 ? s0 : s1, bj = s0 < s1 ? s1 : s0;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int lr = 4 * ks + kg;
            const int row = ks < KS / 2 ? bi * RB + lr : bj * RB + (lr - RB);
            rk[ks] = row < p ? row * lds : -1;
        }
    }
#pragma unroll
    for (int tm = 0; tm < 2; ++tm)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const int row = blk[hw] * RB + tm * 16 + 4 * rr + kg;   // FP64 MFMA accumulator row
            ro[tm][rr] = row < p ? row * ldd : -1;
        }
    const int cb = chunk * GC, ce = min(q, cb + GC);
    const int nsl = (ce - cb + SW - 1) / SW;
    // Gram tiles of this wavefront: w, w + 8 (of the NTILE tiles I <= J)
    int ti[GTW], tj[GTW];
#pragma unroll
    for (int i = 0; i < GTW; ++i) {
        int I = 0, J = w + 8 * i;
        while (J >= NTL - I && I < NTL) {
            J -= NTL - I;
            ++I;
        }
        ti[i] = I;
        tj[i] = J + I;
    }
    d4_t gacc[GTW];
#pragma unroll
    for (int i = 0; i < GTW; ++i) gacc[i] = d4_t{0, 0, 0, 0};
    // Data operands one slice ahead: the loads of slice sl + 1 are issued
    // right after the products of slice sl, into the registers those
    // products consumed, and unconditionally (an out-of-range operand reads
    // element 0 and is replaced by zero where it is used; past the last slice
    // they reread element 0), so that the wait before each slice's products
    // covers exactly that slice's loads.
    double b[KS];
    {
        const int c = cb + csl * 16 + l16;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) b[ks] = Xs[(rk[ks] >= 0 && c < ce) ? rk[ks] + c : 0];
    }
    asm volatile("" ::: "memory");   // keeps the loads above from being moved down to their uses
#pragma unroll
    for (int u = 0; u < QPT; ++u) {
        const int e = t + 512 * u;
        Qh[e / (PR * RB)][(e / RB) % PR][e % RB] = qv[u];
    }
    __syncthreads();
    // this wavefront's Q operands stay in registers for every slice
    double qa[KS][2];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int tm = 0; tm < 2; ++tm) {
            qa[ks][tm] = Qh[hw][4 * ks + kg][tm * 16 + l16];
            asm volatile("" : "+v"(qa[ks][tm]));   // held in registers, not reread from LDS per slice
        }
    for (int sl = 0; sl < nsl; ++sl) {
        const int c = cb + sl * SW + csl * 16 + l16;
        d4_t acc[2] = {d4_t{0, 0, 0, 0}, d4_t{0, 0, 0, 0}};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const double bv = (rk[ks] >= 0 && c < ce) ? b[ks] : 0.0;
#pragma unroll
            for (int tm = 0; tm < 2; ++tm)
                acc[tm] = __builtin_amdgcn_mfma_f64_16x16x4f64(qa[ks][tm], bv, acc[tm], 0, 0, 0);
        }
        {
            const int cn = c + SW;
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) b[ks] = Xs[(rk[ks] >= 0 && cn < ce) ? rk[ks] + cn : 0];
        }
#pragma unroll
        for (int tm = 0; tm < 2; ++tm)
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const bool in = ro[tm][rr] >= 0 && c < ce;
                if (in) Xd[ro[tm][rr] + c] = acc[tm][rr];
                Ys[sl & 1][hw * RB + tm * 16 + 4 * rr + kg][csl * 16 + l16] = in ? acc[tm][rr] : 0.0;
            }
        // one barrier per slice: a wavefront writes the other buffer next,
        // which every wavefront finished reading before reaching this barrier
        __syncthreads();
        const auto& Y = Ys[sl & 1];
        // per tile: all operands read from LDS first, then two independent
        // accumulation chains (even and odd k steps)
#pragma unroll
        for (int i = 0; i < GTW; ++i) {
            if (w + 8 * i >= NTILE) break;
            double ya[SW / 4], yb[SW / 4];
#pragma unroll
            for (int k = 0; k < SW / 4; ++k) {
                ya[k] = Y[ti[i] * 16 + l16][4 * k + kg];
                yb[k] = Y[tj[i] * 16 + l16][4 * k + kg];
            }
            d4_t g2[2] = {d4_t{0, 0, 0, 0}, d4_t{0, 0, 0, 0}};
#pragma unroll
            for (int k = 0; k < SW / 4; ++k) g2[k & 1] = __builtin_amdgcn_mfma_f64_16x16x4f64(ya[k], yb[k], g2[k & 1], 0, 0, 0);
            gacc[i] += g2[0] + g2[1];
        }
    }
    double* out = gram + ((long)Pn * nchunks + chunk) * (PR * PR);
#pragma unroll
    for (int i = 0; i < GTW; ++i) {
        if (w + 8 * i >= NTILE) break;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) out[(ti[i] * 16 + 4 * rr + kg) * PR + tj[i] * 16 + l16] = gacc[i][rr];
    }
}

// Convergence check over all row pairs at once, in place of a sweep that
// would only confirm convergence: with G = X X^T (n x n, leading dimension
// ldg) of the current rows, the largest orthogonality measure over i < j
// (the measure and rounding floor of pair_sweep, sigma1^2 = the larger of
// sigma1sq and the largest diagonal entry).  out[0]: the measure (atomic
// maximum, cleared by the caller), out[1]: the largest diagonal entry.
__global__ __launch_bounds__(256) void gram_diag_kernel(const double* __restrict__ G, int n, long ldg,
                                                        double* __restrict__ diag, double* __restrict__ out) {
    __shared__ double red[4];
    const int j = blockIdx.x * 256 + threadIdx.x;
    const double v = j < n ? fmax(G[(long)j * ldg + j], 0.0) : 0.0;
    if (j < n) diag[j] = v;
    const double m = wave_max_nonneg(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) atomic_max_pos(out + 1, fmax(fmax(red[0], red[1]), fmax(red[2], red[3])));
}

__global__ __launch_bounds__(256) void gram_off_kernel(const double* __restrict__ G, int n, long ldg,
                                                       const double* __restrict__ diag, double kappa,
                                                       double sigma1sq, double* __restrict__ out) {
    __shared__ double red[4];
    const int i = blockIdx.x, t = threadIdx.x;
    const double kappa_s1 = kappa * sqrt(fmax(sigma1sq, out[1]));
    const double gii = diag[i];
    double off = 0.0;
    for (int j = i + 1 + t; j < n; j += 256) {
        const double den = off_den(gii, diag[j], kappa_s1);
        if (den > 0.0) off = fmax(off, fabs(G[(long)i * ldg + j]) / den);
    }
    off = wave_max_nonneg(off);
    if ((t & 63) == 0) red[t >> 6] = off;
    __syncthreads();
    if (t == 0) atomic_max_pos(out, fmax(fmax(red[0], red[1]), fmax(red[2], red[3])));
}

// Dst[i][c] = Src[i][c] for i < p, c < q (data columns back to the work matrix).
__global__ void copy_cols_kernel(const double* __restrict__ src, int lds, double* __restrict__ dst, int ldd, int p,
                                 int q) {
    const long total = (long)p * q;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
        const int i = (int)(e / q), c = (int)(e % q);
        dst[(long)i * ldd + c] = src[(long)i * lds + c];
    }
}

// Rotation of columns [cb, ce) for the pairs of round r, cw columns per
// workgroup (grid: column chunks x pairs).  Pairs without rotation skip.
// work counts the columns rotated.
// Eight wavefronts per workgroup with Q read from LDS for every slice (two
// wavefronts per SIMD) measured faster than four holding Q in registers.
constexpr int ROT_WAVES = 8;
template <int RB>
__global__ __launch_bounds__(64 * ROT_WAVES) void rotate_kernel(double* __restrict__ Z, int p, int ld, int r, int nb,
                                                     const double* __restrict__ rot,
                                                     const int* __restrict__ rotated, int cb, int ce, int cw,
                                                     unsigned long long* __restrict__ work) {
    constexpr int PR = Blk<RB>::PR;
    const int P = blockIdx.y;
    if (!rotated[P]) return;
    const int c0 = cb + blockIdx.x * cw, c1 = min(c0 + cw, ce);
    if (threadIdx.x == 0) atomicAdd(work, (unsigned long long)(c1 - c0));
    __shared__ double Qs[PR][PR + 1];        // Q[k][m]
    const double* src = rot + (long)P * PR * PR;
    for (int e = threadIdx.x; e < PR * PR; e += 64 * ROT_WAVES) Qs[e / PR][e % PR] = src[e];
    rotate_cols<RB, ROT_WAVES, true, false>(Z, p, ld, P, r, nb, Qs, c0, c1, threadIdx.x, true);
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

template <int RB>
void ws_sizes(int p, int q, size_t* gram, size_t* rot, size_t* off) {
    constexpr int PR = Blk<RB>::PR, GC = Blk<RB>::GC;
    int nb = (p + RB - 1) / RB;
    if (nb < 2) nb = 2;
    if (nb & 1) ++nb;
    const size_t npairs = nb / 2, nchunks = std::max(1, (q + GC - 1) / GC);
    // Gram partials, then (32-row blocks) the second buffer of the data columns
    *gram = npairs * nchunks * PR * PR + (RB == 32 ? (size_t)p * q : 0);
    *rot = 2 * npairs * PR * PR;     // rotations of two consecutive rounds
    *off = npairs + 24 + (size_t)p;     // flags, counters, check result, Gram diagonal
}

// Columns per rotate workgroup: wide chunks amortise the load of Q, narrow
// ones give the launch enough workgroups to fill the chip.
inline int rotate_width(int npairs, int ncols) {
    int cw = 512;
    while (cw > 128 && (long)npairs * ((ncols + cw - 1) / cw) < 256) cw /= 2;
    return cw;
}

template <int RB>
JacobiResult run_jacobi(double* Z, int p, int q, int ld, double tol, int max_sweeps, double* gram_ws,
                        double* rot_ws, double* off_ws, double* host_off, hipStream_t s, LaunchProbe* probe) {
    constexpr int GC = Blk<RB>::GC, NT = Blk<RB>::NT, PR = Blk<RB>::PR, UW = Blk<RB>::UW;
    JacobiResult res;
    int nb = (p + RB - 1) / RB;
    if (nb < 2) nb = 2;
    if (nb & 1) ++nb;
    const int npairs = nb / 2;
    const int nchunks = std::max(1, (q + GC - 1) / GC);
    const int nu = ld - q;                         // identity-part columns
    const int nuch = (nu + UW - 1) / UW;
    // off_ws[0]: largest off-diagonal measure of the sweep, off_ws[1]: largest
    // row norm squared seen in it, then the rotated flags of two consecutive
    // rounds (npairs ints each), then five work counters (gram chunks, inner
    // pairs, columns rotated by rotate launches, identity-part columns
    // rotated by inner launches, data columns rotated by fused launches)
    int* rotated = reinterpret_cast<int*>(off_ws + 2);
    unsigned long long* work = reinterpret_cast<unsigned long long*>(off_ws + 2 + npairs);
    if (probe) fill(off_ws + 2 + npairs, 0.0, 5, s);
    // 32-row blocks: the rotation of round r and the Gram of round r + 1 are
    // one launch, whose new data rows go to the other of two buffers (the Z
    // columns 0..q and Xb); round g reads buffer g mod 2
    static_assert(RB == 32, "the multi-pair rounds use 32-row blocks and the fused rotation + Gram");
    double* Xb = gram_ws + (size_t)npairs * nchunks * PR * PR;
    {
        bool timed = probe && probe->begin(PK_GRAM, s);
        hipLaunchKernelGGL((gram_kernel<RB>), dim3(nchunks, npairs), dim3(GRAM_NT), 0, s, Z, p, q, ld, 0, nb,
                           nchunks, gram_ws, work);
        if (timed) probe->end(PK_GRAM, s);
    }
    constexpr double kappa = 1e-3;
    double prev = 1e300, sigma1sq = 0.0;
    int checks = 0;
    // The identity part of round g's rotations is applied during round
    // g + 1 (by the extra workgroups of its inner launch) and after the last
    // round; rotations and flags alternate between two buffers.
    long g = 0;
    int rprev = -1;
    for (int sw = 0; sw < max_sweeps; ++sw) {
        fill(off_ws, 0.0, 2, s);
        // far from convergence the pair sweeps rotate a single-precision copy
        // of the Gram (the measure and the accumulated rotation stay FP64):
        // their angles only need to be roughly right while the measure is
        // large, and the sweeps that reach the tolerance run in FP64
        const bool lowg = prev > 1e-3;
        for (int r = 0; r < nb - 1; ++r, ++g) {
            const int cur = (int)(g & 1);
            double* rcur = rot_ws + (long)cur * npairs * PR * PR;
            const double* rold = rot_ws + (long)(cur ^ 1) * npairs * PR * PR;
            int* fcur = rotated + cur * npairs;
            const int* fold = rotated + (cur ^ 1) * npairs;
            bool timed = probe && probe->begin(PK_INNER, s);
            const int ublocks = (rprev >= 0 && nu > 0) ? npairs * nuch : 0;
            if (lowg)
                hipLaunchKernelGGL((inner_kernel<RB, float>), dim3(npairs + ublocks), dim3(Blk<RB>::NTI), 0, s,
                                   gram_ws, nchunks, p, r, nb, tol, kappa, sigma1sq, rcur, fcur, off_ws, work, Z, ld,
                                   q, npairs, rprev, rold, fold, nuch);
            else
                hipLaunchKernelGGL((inner_kernel<RB, double>), dim3(npairs + ublocks), dim3(Blk<RB>::NTI), 0, s,
                                   gram_ws, nchunks, p, r, nb, tol, kappa, sigma1sq, rcur, fcur, off_ws, work, Z, ld,
                                   q, npairs, rprev, rold, fold, nuch);
            if (timed) probe->end(PK_INNER, s);
            timed = probe && probe->begin(PK_ROTATE, s);
            {
                const bool odd = g & 1;
                hipLaunchKernelGGL((rotate_gram_kernel<RB>), dim3(nchunks, npairs), dim3(512), 0, s,
                                   odd ? Xb : Z, odd ? q : ld, odd ? Z : Xb, odd ? ld : q, p, q, r, nb, nchunks, rcur,
                                   gram_ws, work + 4);
            }
            if (timed) probe->end(PK_ROTATE, s);
            rprev = r;
        }
        HIP_CHECK(hipGetLastError());
        HIP_CHECK(hipMemcpyAsync(host_off, off_ws, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        const double soff = host_off[0];
        sigma1sq = host_off[1];
        res.sweeps = sw + 1;
        res.last_off = soff;
        if (soff <= tol) break;
        // In the quadratic phase the next sweep would most likely only
        // confirm convergence: check all row pairs at once instead, with the
        // Gram of the current rows formed in the free data buffer (at most
        // two checks per split)
        if (p <= q && soff < 1e-6 && checks < 2) {
            ++checks;
            const bool odd = g & 1;                    // the rows are in Xb when odd
            const double* X = odd ? Xb : Z;
            const long ldx = odd ? q : ld;
            double* G = odd ? Z : Xb;
            const long ldg = odd ? ld : p;
            double* chk = off_ws + 2 + npairs + 8;
            double* diag = chk + 8;
            const bool timed = probe && probe->begin(PK_GRAM, s);
            Gemm gm;
            gm.M = p;
            gm.N = p;
            gm.K = q;
            gm.tB = true;
            gm.A = X;
            gm.lda = ldx;
            gm.B = X;
            gm.ldb = ldx;
            gm.D = G;
            gm.ldd = ldg;
            gemm_f64(gm, s);
            fill(chk, 0.0, 2, s);
            hipLaunchKernelGGL(gram_diag_kernel, dim3((p + 255) / 256), dim3(256), 0, s, G, p, ldg, diag, chk);
            hipLaunchKernelGGL(gram_off_kernel, dim3(p), dim3(256), 0, s, G, p, ldg, diag, kappa, sigma1sq, chk);
            if (timed) probe->end(PK_GRAM, s);
            HIP_CHECK(hipGetLastError());
            HIP_CHECK(hipMemcpyAsync(host_off, chk, sizeof(double), hipMemcpyDeviceToHost, s));
            HIP_CHECK(hipStreamSynchronize(s));
            if (*host_off <= tol) {
                res.last_off = *host_off;
                break;
            }
        }
        // stagnation at the rounding floor: stop once the measure no longer drops
        if (sw >= 3 && soff > 0.5 * prev && soff < 1e3 * tol) break;
        prev = soff;
    }
    if (g & 1) {
        // the final data rows are in Xb
        const long total = (long)p * q;
        hipLaunchKernelGGL(copy_cols_kernel, dim3((int)std::min<long>(4096, (total + 255) / 256)), dim3(256), 0, s, Xb,
                           q, Z, ld, p, q);
        HIP_CHECK(hipGetLastError());
    }
    if (rprev >= 0 && nu > 0) {
        // identity part of the last round
        const int cur = (int)((g - 1) & 1);
        const int uw = rotate_width(npairs, nu);
        bool timed = probe && probe->begin(PK_ROTATE, s);
        hipLaunchKernelGGL((rotate_kernel<RB>), dim3((nu + uw - 1) / uw, npairs), dim3(64 * ROT_WAVES), 0, s, Z, p, ld, rprev,
                           nb, rot_ws + (long)cur * npairs * PR * PR, rotated + cur * npairs, q, ld, uw, work + 2);
        if (timed) probe->end(PK_ROTATE, s);
        HIP_CHECK(hipGetLastError());
    }
    if (probe) {
        // algorithmic work actually done: a chunk Gram is 2 PR^2 GC flops over
        // PR GC doubles read; a pair's inner sweep applies PR (PR - 1) / 2
        // rotations to two rows and two columns of G and two rows of Q
        // (18 PR flops each) plus the Newton-Schulz step (4 PR^3); a rotated
        // column is 2 PR^2 flops over 2 PR doubles read and written (the
        // identity-part columns rotated inside inner launches count there);
        // a fused column also forms the next round's Gram tiles (1.25 PR^2
        // flops, 10 tiles of 256 doubles written per GC columns); the check
        // of all row pairs is one p x p x q product over the rows read once
        unsigned long long cnt[5];
        HIP_CHECK(hipMemcpyAsync(cnt, work, sizeof(cnt), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        const double pr = PR;
        (void)NT;
        probe->work(PK_GRAM, cnt[0] * 2.0 * pr * pr * GC + checks * 2.0 * p * p * q,
                    cnt[0] * 8.0 * pr * GC + checks * 8.0 * ((double)p * q + (double)p * p));
        probe->work(PK_INNER, cnt[1] * (9.0 * pr * pr * (pr - 1) + 4.0 * pr * pr * pr) + cnt[3] * 2.0 * pr * pr,
                    cnt[1] * 8.0 * 2 * pr * pr + cnt[3] * 16.0 * pr);
        probe->work(PK_ROTATE, cnt[2] * 2.0 * pr * pr + cnt[4] * 3.25 * pr * pr,
                    cnt[2] * 16.0 * pr + cnt[4] * (16.0 * pr + 8.0 * 10 * 256 / GC));
    }
    return res;
}

}  // namespace

void jacobi_workspace(int p, int q, size_t* gram, size_t* rot, size_t* off) {
    ws_sizes<32>(p, q, gram, rot, off);
}

JacobiResult jacobi_rows(double* Z, int p, int q, int ld, double tol, int max_sweeps, double* gram_ws,
                         double* rot_ws, double* off_ws, double* host_off, hipStream_t s, LaunchProbe* probe) {
    if (p <= 1) return JacobiResult{};
    ITE_REQUIRE((long)p * ld < 2147483647L, "svd: work matrix too large for 32-bit element offsets");
    if (p <= Blk<32>::PR) {
        // one block pair: the whole Jacobi in one launch and one host read
        bool timed = probe && probe->begin(PK_INNER, s);
        if (p <= Blk<16>::PR)
            hipLaunchKernelGGL((single_pair_jacobi_kernel<16>), dim3(1), dim3(Blk<16>::NTI), 0, s, Z, p, q, ld, tol,
                               1e-3, max_sweeps, off_ws);
        else
            hipLaunchKernelGGL((single_pair_jacobi_kernel<32>), dim3(1), dim3(Blk<32>::NTI), 0, s, Z, p, q, ld, tol,
                               1e-3, max_sweeps, off_ws);
        if (timed) probe->end(PK_INNER, s);
        HIP_CHECK(hipGetLastError());
        HIP_CHECK(hipMemcpyAsync(host_off, off_ws, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        JacobiResult res;
        res.last_off = host_off[0];
        res.sweeps = (int)host_off[1];
        if (probe) {
            // per sweep: the Gram (p^2 q flops), the inner sweep of the pair and the
            // rotation of p rows over ld columns
            const double pr = p <= Blk<16>::PR ? Blk<16>::PR : Blk<32>::PR, sw = res.sweeps;
            probe->work(PK_INNER, sw * (2.0 * p * p * q + 9.0 * pr * pr * (pr - 1) + 4.0 * pr * pr * pr + 2.0 * p * p * ld),
                        sw * 8.0 * (double)p * (q + 2.0 * ld));
        }
        return res;
    }
    return run_jacobi<32>(Z, p, q, ld, tol, max_sweeps, gram_ws, rot_ws, off_ws, host_off, s, probe);
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
