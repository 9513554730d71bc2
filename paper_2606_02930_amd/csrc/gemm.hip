// Tiled MFMA GEMM for gfx950 (CDNA4): the contraction core of the
// effective-Hamiltonian product and of the environment updates.
//
// D[b] = alpha op(A[b]) op(B[b]) + beta C[b], row-major.
//
// Tile: 128 x 128 output per workgroup of 256 threads (four 64-wide
// wavefronts in a 2 x 2 arrangement, each owning 64 x 64 = 4 x 4 MFMA tiles of
// 16 x 16).  Registers are kept within 256 per lane (operands of two MFMA
// sub-steps live at a time) so that two workgroups share a CU and one's
// barrier and LDS traffic overlap the other's matrix-core work.  K advances in slices of 16 staged through LDS with double
// buffering: the next slice is fetched into registers while the current one
// feeds the matrix cores.  Both operands are stored in LDS "K-contiguous"
// (row = output row or column, 16 K values per row, padded) so that each lane
// fetches its four K values for the four MFMA sub-steps of a slice with two
// 16-byte LDS reads.  Within a slice, lane group g = lane / 16 supplies K
// index 4 g + step in sub-step `step`; A and B use the same mapping, so the
// sum over K is unchanged.
//
// Workgroup -> tile mapping is XCD-aware: the hardware deals workgroups to the
// 8 XCDs round-robin, so consecutive workgroup ids are remapped to give each
// XCD a contiguous band of output tiles that share A row panels in that XCD's
// L2.
#include "internal.h"

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <type_traits>

namespace ite {
namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

constexpr int BM = 128;
constexpr int BN = 128;
constexpr int BK = 16;
constexpr int NTHREADS = 256;

template <typename T> struct MfmaOp;
template <> struct MfmaOp<double> {
    typedef d4_t acc_t;
    static constexpr int LDK = BK + 2;   // 144-byte rows: 16-byte aligned, few bank conflicts
    __device__ static acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // tile row of accumulator element r in lane group g = lane / 16
    __device__ static int row(int g, int r) { return 4 * r + g; }
};
template <> struct MfmaOp<float> {
    typedef f4_t acc_t;
    static constexpr int LDK = BK + 4;   // 80-byte rows
    __device__ static acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static int row(int g, int r) { return 4 * g + r; }
};

struct Params {
    int M, N, K;
    double alpha, beta;
    const void* A; long lda, sA;
    const void* B; long ldb, sB;
    const double* C; long ldc, sC;
    double* D; long ldd, sD;
    int mt, nt;
    float* Df;      // FP32 output instead of D (no C)
};

// Bijection from the hardware workgroup id to an output tile such that XCD x
// (workgroups with id % 8 == x) receives a contiguous range of tiles.
__device__ inline int xcd_band_tile(int bid, int T) {
    const int q = T >> 3, r = T & 7;
    const int xcd = bid & 7, idx = bid >> 3;
    const int base = xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q;
    return base + idx;
}

// Stage one K slice of an operand into registers (BS = 128 or 64 rows of the
// tile side, E = BS * 16 / 256 values per thread).  KC: the source is stored
// with K contiguous (rows of the tile side are strided by ld); otherwise K is
// the slow index (rows are K, the tile side is contiguous).
template <typename T, bool KC, int BS>
__device__ inline void fetch_slice(const T* __restrict__ src, long ld, int side0, int sideN, int k0,
                                   int K, int t, T (&r)[BS / 16]) {
    constexpr int E = BS / 16;
    if (KC) {
        const int kk = t & 15;
        const int k = k0 + kk;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int row = side0 + (t >> 4) + 16 * e;
            r[e] = (row < sideN && k < K) ? src[(long)row * ld + k] : T(0);
        }
    } else {
        const int col = side0 + (t % BS);
        const int kh = (t / BS) * E;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = k0 + kh + e;
            r[e] = (col < sideN && k < K) ? src[(long)k * ld + col] : T(0);
        }
    }
}

template <typename T, bool KC, int BS>
__device__ inline void store_slice(T* __restrict__ lds, int t, const T (&r)[BS / 16]) {
    constexpr int LDK = MfmaOp<T>::LDK, E = BS / 16;
    if (KC) {
        const int kk = t & 15;
#pragma unroll
        for (int e = 0; e < E; ++e) lds[((t >> 4) + 16 * e) * LDK + kk] = r[e];
    } else {
        const int row = t % BS;
        const int kh = (t / BS) * E;
#pragma unroll
        for (int e = 0; e < E; ++e) lds[row * LDK + kh + e] = r[e];
    }
}

// 16-byte loads of a 128-wide FP32 operand slice (four floats each) into
// the same registers and LDS layout as fetch_slice / store_slice, so the
// products are the same; chunks that cross the matrix edge are loaded
// element by element.  Needs 16-byte aligned rows (checked by the launcher).
template <bool KC>
__device__ inline void fetch_slice_v4(const float* __restrict__ src, long ld, int side0, int sideN, int k0, int K,
                                      int t, float (&r)[8]) {
    if (KC) {
        const int row = side0 + (t >> 1);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int k = k0 + (t & 1) * 8 + 4 * c;
            if (row < sideN && k + 3 < K) {
                const float4 v = *reinterpret_cast<const float4*>(src + (long)row * ld + k);
                r[4 * c] = v.x; r[4 * c + 1] = v.y; r[4 * c + 2] = v.z; r[4 * c + 3] = v.w;
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) r[4 * c + q] = (row < sideN && k + q < K) ? src[(long)row * ld + k + q] : 0.f;
            }
        }
    } else {
        const int col = side0 + (t & 31) * 4;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int k = k0 + (t >> 5) + 8 * e;
            if (k < K && col + 3 < sideN) {
                const float4 v = *reinterpret_cast<const float4*>(src + (long)k * ld + col);
                r[4 * e] = v.x; r[4 * e + 1] = v.y; r[4 * e + 2] = v.z; r[4 * e + 3] = v.w;
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) r[4 * e + q] = (k < K && col + q < sideN) ? src[(long)k * ld + col + q] : 0.f;
            }
        }
    }
}

template <bool KC>
__device__ inline void store_slice_v4(float* __restrict__ lds, int t, const float (&r)[8]) {
    constexpr int LDK = MfmaOp<float>::LDK;
    if (KC) {
        const int row = t >> 1;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int kk = (t & 1) * 8 + 4 * c;
            *reinterpret_cast<float4*>(&lds[row * LDK + kk]) = make_float4(r[4 * c], r[4 * c + 1], r[4 * c + 2], r[4 * c + 3]);
        }
    } else {
        const int col = (t & 31) * 4;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int krow = (t >> 5) + 8 * e;
#pragma unroll
            for (int q = 0; q < 4; ++q) lds[(col + q) * LDK + krow] = r[4 * e + q];
        }
    }
}

// The operand slice loaders of gemm_tile: 16-byte loads for FP32 operands
// of the 128 tile when VEC, the element loads otherwise.
template <typename T, bool KC, int BS, bool VEC>
__device__ inline void fetch_op(const T* __restrict__ src, long ld, int side0, int sideN, int k0, int K, int t,
                                T (&r)[BS / 16]) {
    if constexpr (VEC && std::is_same<T, float>::value && BS == 128) fetch_slice_v4<KC>(src, ld, side0, sideN, k0, K, t, r);
    else fetch_slice<T, KC, BS>(src, ld, side0, sideN, k0, K, t, r);
}
template <typename T, bool KC, int BS, bool VEC>
__device__ inline void store_op(T* __restrict__ lds, int t, const T (&r)[BS / 16]) {
    if constexpr (VEC && std::is_same<T, float>::value && BS == 128) store_slice_v4<KC>(lds, t, r);
    else store_slice<T, KC, BS>(lds, t, r);
}

// One BS x BS output tile at (m0, n0) of problem p (batch index bz): four
// wavefronts in a 2 x 2 arrangement, each owning (BS / 2)^2 outputs as
// (BS / 32)^2 MFMA tiles of 16 x 16.  The K order of every output element
// (slices of 16, four sub-steps, lane group g supplying K index 4 g + step)
// does not depend on BS, so the 128 and 64 tiles give the same bits.  As, Bs:
// LDS of two slices of each operand.  Ends with a barrier after the last LDS
// read, so the caller may start another tile.
template <typename T, bool TA, bool TB, int BS, bool VEC = false>
__device__ __forceinline__ void gemm_tile(const Params& p, int m0, int n0, long bz, T* As, T* Bs) {
    typedef typename MfmaOp<T>::acc_t acc_t;
    constexpr int LDK = MfmaOp<T>::LDK, IT = BS / 32, E = BS / 16;
    const T* __restrict__ A = static_cast<const T*>(p.A) + bz * p.sA;
    const T* __restrict__ B = static_cast<const T*>(p.B) + bz * p.sB;

    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = t >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int l16 = lane & 15, kg = lane >> 4;

    acc_t acc[IT][IT];
#pragma unroll
    for (int i = 0; i < IT; ++i)
#pragma unroll
        for (int j = 0; j < IT; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

    // A: K-contiguous unless transposed.  B: K-contiguous only when transposed.
    T ra[E], rb[E];
    const int nk = (p.K + BK - 1) / BK;
    fetch_op<T, !TA, BS, VEC>(A, p.lda, m0, p.M, 0, p.K, t, ra);
    fetch_op<T, TB, BS, VEC>(B, p.ldb, n0, p.N, 0, p.K, t, rb);
    store_op<T, !TA, BS, VEC>(As, t, ra);
    store_op<T, TB, BS, VEC>(Bs, t, rb);
    __syncthreads();

    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        const bool more = kt + 1 < nk;
        const T* Ac = As + cur * BS * LDK;
        const T* Bc = Bs + cur * BS * LDK;
        if (more) {
            fetch_op<T, !TA, BS, VEC>(A, p.lda, m0, p.M, (kt + 1) * BK, p.K, t, ra);
            fetch_op<T, TB, BS, VEC>(B, p.ldb, n0, p.N, (kt + 1) * BK, p.K, t, rb);
        }
        // two sub-steps of the slice at a time: 16 operand values live
        // instead of 32, which leaves room for two workgroups per CU
#pragma unroll
        for (int s2 = 0; s2 < 4; s2 += 2) {
            T a[IT][2], b[IT][2];
#pragma unroll
            for (int i = 0; i < IT; ++i) {
                const T* src = &Ac[(wm * (BS / 2) + i * 16 + l16) * LDK + 4 * kg + s2];
                a[i][0] = src[0];
                a[i][1] = src[1];
            }
#pragma unroll
            for (int j = 0; j < IT; ++j) {
                const T* src = &Bc[(wn * (BS / 2) + j * 16 + l16) * LDK + 4 * kg + s2];
                b[j][0] = src[0];
                b[j][1] = src[1];
            }
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int i = 0; i < IT; ++i)
#pragma unroll
                    for (int j = 0; j < IT; ++j) acc[i][j] = MfmaOp<T>::mma(a[i][s], b[j][s], acc[i][j]);
        }
        if (more) {
            store_op<T, !TA, BS, VEC>(As + (cur ^ 1) * BS * LDK, t, ra);
            store_op<T, TB, BS, VEC>(Bs + (cur ^ 1) * BS * LDK, t, rb);
        }
        __syncthreads();
    }

    // Epilogue.  Accumulator element r of lane l holds column l % 16 of its
    // 16 x 16 tile and row 4 r + l / 16 (FP64 MFMA) or 4 (l / 16) + r (FP32).
    const double* __restrict__ C = p.C ? p.C + bz * p.sC : nullptr;
    double* __restrict__ D = p.Df ? nullptr : p.D + bz * p.sD;
    float* __restrict__ Df = p.Df ? p.Df + bz * p.sD : nullptr;
#pragma unroll
    for (int i = 0; i < IT; ++i)
#pragma unroll
        for (int j = 0; j < IT; ++j) {
            const int col = n0 + wn * (BS / 2) + j * 16 + l16;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm * (BS / 2) + i * 16 + MfmaOp<T>::row(kg, r);
                if (row < p.M && col < p.N) {
                    double v = p.alpha * (double)acc[i][j][r];
                    if (Df) {
                        Df[(long)row * p.ldd + col] = (float)v;
                    } else {
                        if (C) v += p.beta * C[(long)row * p.ldc + col];
                        D[(long)row * p.ldd + col] = v;
                    }
                }
            }
        }
}

template <typename T, bool TA, bool TB, bool VEC = false>
__global__ __launch_bounds__(NTHREADS, 2) void gemm_kernel(Params p) {
    constexpr int LDK = MfmaOp<T>::LDK;
    __shared__ __attribute__((aligned(16))) T As[2 * BM * LDK];
    __shared__ __attribute__((aligned(16))) T Bs[2 * BN * LDK];
    const int T_tiles = p.mt * p.nt;
    const int tile = xcd_band_tile(blockIdx.x, T_tiles);
    const int m0 = (tile / p.nt) * BM;
    const int n0 = (tile % p.nt) * BN;
    gemm_tile<T, TA, TB, BM, VEC>(p, m0, n0, (long)blockIdx.z, As, Bs);
}

// Many independent FP64 problems in one persistent launch (the products of
// the requests batched by the serving path): problem g's tiles are
// [tile_start[g], tile_start[g + 1]) of a common range, row-major over its
// output; every workgroup walks that range with a stride of the grid, so the
// grid can stay fixed (graph capture) while the problems change.  The
// descriptors live in device memory; BS as gemm_tile.
struct GroupDesc {
    Params p;
    int tile_start;
};

template <typename T, bool TA, bool TB, int BS>
__global__ __launch_bounds__(NTHREADS, 2) void gemm_grouped_kernel(const GroupDesc* __restrict__ desc,
                                                                   const int* __restrict__ count) {
    constexpr int LDK = MfmaOp<T>::LDK;
    __shared__ __attribute__((aligned(16))) T As[2 * BS * LDK];
    __shared__ __attribute__((aligned(16))) T Bs[2 * BS * LDK];
    const int G = count[0], ntiles = count[1];
    int g = 0;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        while (g + 1 < G && desc[g + 1].tile_start <= tile) ++g;
        const Params& p = desc[g].p;
        const int lt = tile - desc[g].tile_start;
        gemm_tile<T, TA, TB, BS>(p, (lt / p.nt) * BS, (lt % p.nt) * BS, 0, As, Bs);
    }
}

// Operands fit 16-byte loads: aligned bases, row strides and batch strides
// that are multiples of 16 bytes.
inline bool vec16(const Gemm& g, size_t esz) {
    const size_t q = 16 / esz;
    auto al = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
    return al(g.A) && al(g.B) && g.lda % q == 0 && g.ldb % q == 0 && g.sA % q == 0 && g.sB % q == 0;
}

template <typename T>
void launch(const Gemm& g, hipStream_t s) {
    if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return;
    if (g.Df && g.C) ITE_FAIL(ITE_EINVAL, "gemm: an FP32 output takes no C");
    Params p;
    p.M = g.M; p.N = g.N; p.K = g.K;
    p.alpha = g.alpha; p.beta = g.beta;
    p.A = g.A; p.lda = g.lda; p.sA = g.sA;
    p.B = g.B; p.ldb = g.ldb; p.sB = g.sB;
    p.C = g.C; p.ldc = g.ldc; p.sC = g.sC;
    p.D = g.D; p.ldd = g.ldd; p.sD = g.sD;
    p.Df = std::is_same<T, float>::value ? g.Df : nullptr;
    p.mt = (g.M + BM - 1) / BM;
    p.nt = (g.N + BN - 1) / BN;
    dim3 grid(p.mt * p.nt, 1, g.batch);
    const bool v = std::is_same<T, float>::value && vec16(g, sizeof(T));
#define ITE_GL(TA, TB)                                                                              \
    if (v) hipLaunchKernelGGL((gemm_kernel<T, TA, TB, true>), grid, dim3(NTHREADS), 0, s, p);       \
    else hipLaunchKernelGGL((gemm_kernel<T, TA, TB, false>), grid, dim3(NTHREADS), 0, s, p)
    if (!g.tA && !g.tB) { ITE_GL(false, false); }
    else if (!g.tA && g.tB) { ITE_GL(false, true); }
    else if (g.tA && !g.tB) { ITE_GL(true, false); }
    else { ITE_GL(true, true); }
#undef ITE_GL
    HIP_CHECK(hipGetLastError());
}

// One v_mfma_f64_16x16x4f64 with A[i][k] = 1 + i + 16 k (i < 16, k < 4)
// supplied by lane i + 16 k and B[k][j] = 1 / (1 + j + 16 k) by lane j + 16 k;
// every lane writes its four accumulator values.
__global__ void mfma_probe_kernel(double* out) {
    const int l = threadIdx.x;
    const double a = 1.0 + (l & 15) + 16.0 * (l >> 4);
    const double b = 1.0 / (1.0 + (l & 15) + 16.0 * (l >> 4));
    d4_t acc = {0, 0, 0, 0};
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    for (int r = 0; r < 4; ++r) out[l * 4 + r] = acc[r];
}

// ---------------------------------------------------------------------------
// BF16 operands, FP32 accumulation: v_mfma_f32_16x16x32_bf16 (gfx950).  Same
// 128 x 128 tile and 2 x 2 wave arrangement as above; K advances in slices of
// 64 (two MFMA K steps per 16 x 16 tile, 32 MFMAs per wave between barriers).
// Both operands sit in LDS as [row][64 K values] (row = output row or
// column), in 16-byte chunks of 8 K values whose position within the row is
// XOR-swizzled by the row index, so that the MFMA reads (16 rows, one chunk
// each) and the transposing writes of a side-contiguous operand spread over
// the banks without padding.  Lane group g = lane / 16 supplies K values
// 8 g .. 8 g + 7 of each 32-wide step; A and B use the same mapping.
// ---------------------------------------------------------------------------
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
constexpr int BK16 = 64;

// u16 offset of chunk c (8 K values) of LDS row r
__device__ inline int swz16(int r, int c) { return r * BK16 + ((c ^ (r & 7) ^ ((r >> 3) & 7)) << 3); }

// Registers of one operand's K slice: four 16-byte words per thread.
struct Slice16 {
    uint4 v[4];
};

// K-contiguous source ([side][K]): thread t fetches chunks u = t + 256 e,
// row u / 8, chunk u % 8 (eight threads read one row's 128 bytes).
template <bool VEC>
__device__ inline void fetch16_kc(const uint16_t* __restrict__ src, long ld, int side0, int sideN, int k0, int K,
                                  int t, Slice16& r) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int u = t + 256 * e;
        const int row = side0 + (u >> 3);
        const int k = k0 + (u & 7) * 8;
        if (VEC && row < sideN && k + 7 < K) {
            r.v[e] = *reinterpret_cast<const uint4*>(src + (long)row * ld + k);
        } else {
            uint16_t h[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) h[q] = (row < sideN && k + q < K) ? src[(long)row * ld + k + q] : (uint16_t)0;
            r.v[e] = uint4{(uint32_t)h[0] | ((uint32_t)h[1] << 16), (uint32_t)h[2] | ((uint32_t)h[3] << 16),
                           (uint32_t)h[4] | ((uint32_t)h[5] << 16), (uint32_t)h[6] | ((uint32_t)h[7] << 16)};
        }
    }
}
__device__ inline void store16_kc(uint16_t* __restrict__ lds, int t, const Slice16& r) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int u = t + 256 * e;
        *reinterpret_cast<uint4*>(&lds[swz16(u >> 3, u & 7)]) = r.v[e];
    }
}

// Side-contiguous source ([K][side]): thread t fetches a 4 (K) x 8 (side)
// block, K rows 4 (t / 16) .. +3 and side values 8 (t % 16) .. +7 (sixteen
// threads read one K row's 256 bytes), and writes it transposed: eight LDS
// rows of four K values (8 bytes each).
template <bool VEC>
__device__ inline void fetch16_sc(const uint16_t* __restrict__ src, long ld, int side0, int sideN, int k0, int K,
                                  int t, Slice16& r) {
    const int col = side0 + (t & 15) * 8;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int k = k0 + (t >> 4) * 4 + e;
        if (VEC && k < K && col + 7 < sideN) {
            r.v[e] = *reinterpret_cast<const uint4*>(src + (long)k * ld + col);
        } else {
            uint16_t h[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) h[q] = (k < K && col + q < sideN) ? src[(long)k * ld + col + q] : (uint16_t)0;
            r.v[e] = uint4{(uint32_t)h[0] | ((uint32_t)h[1] << 16), (uint32_t)h[2] | ((uint32_t)h[3] << 16),
                           (uint32_t)h[4] | ((uint32_t)h[5] << 16), (uint32_t)h[6] | ((uint32_t)h[7] << 16)};
        }
    }
}
__device__ inline uint32_t word16(const uint4& v, int q) {
    const uint32_t w = q < 2 ? (q == 0 ? v.x : v.y) : (q == 2 ? v.z : v.w);
    return w;
}
__device__ inline void store16_sc(uint16_t* __restrict__ lds, int t, const Slice16& r) {
    const int s0 = (t & 15) * 8;
    const int kb = t >> 4;   // K values 4 kb .. 4 kb + 3: chunk kb / 2, half kb % 2
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const uint32_t a0 = word16(r.v[0], w), a1 = word16(r.v[1], w);
        const uint32_t a2 = word16(r.v[2], w), a3 = word16(r.v[3], w);
        // side value 2 w (low halves) and 2 w + 1 (high halves)
        const uint2 lo{(a0 & 0xffffu) | (a1 << 16), (a2 & 0xffffu) | (a3 << 16)};
        const uint2 hi{(a0 >> 16) | (a1 & 0xffff0000u), (a2 >> 16) | (a3 & 0xffff0000u)};
        *reinterpret_cast<uint2*>(&lds[swz16(s0 + 2 * w, kb >> 1) + (kb & 1) * 4]) = lo;
        *reinterpret_cast<uint2*>(&lds[swz16(s0 + 2 * w + 1, kb >> 1) + (kb & 1) * 4]) = hi;
    }
}

template <bool KC, bool VEC>
__device__ inline void fetch16(const uint16_t* __restrict__ src, long ld, int side0, int sideN, int k0, int K, int t,
                               Slice16& r) {
    if constexpr (KC) fetch16_kc<VEC>(src, ld, side0, sideN, k0, K, t, r);
    else fetch16_sc<VEC>(src, ld, side0, sideN, k0, K, t, r);
}
template <bool KC>
__device__ inline void store16(uint16_t* __restrict__ lds, int t, const Slice16& r) {
    if constexpr (KC) store16_kc(lds, t, r);
    else store16_sc(lds, t, r);
}

template <bool TA, bool TB, bool VEC>
__global__ __launch_bounds__(NTHREADS) void gemm_bf16_kernel(Params p) {
    __shared__ __attribute__((aligned(16))) uint16_t As[2][BM * BK16];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[2][BN * BK16];
    const int T_tiles = p.mt * p.nt;
    const int tile = xcd_band_tile(blockIdx.x, T_tiles);
    const int m0 = (tile / p.nt) * BM;
    const int n0 = (tile % p.nt) * BN;
    const long bz = blockIdx.z;
    const uint16_t* __restrict__ A = static_cast<const uint16_t*>(p.A) + bz * p.sA;
    const uint16_t* __restrict__ B = static_cast<const uint16_t*>(p.B) + bz * p.sB;
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = t >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int l16 = lane & 15, kg = lane >> 4;
    f4_t acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f4_t{0, 0, 0, 0};
    Slice16 ra, rb;
    const int nk = (p.K + BK16 - 1) / BK16;
    fetch16<!TA, VEC>(A, p.lda, m0, p.M, 0, p.K, t, ra);
    fetch16<TB, VEC>(B, p.ldb, n0, p.N, 0, p.K, t, rb);
    store16<!TA>(As[0], t, ra);
    store16<TB>(Bs[0], t, rb);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        const bool more = kt + 1 < nk;
        if (more) {
            fetch16<!TA, VEC>(A, p.lda, m0, p.M, (kt + 1) * BK16, p.K, t, ra);
            fetch16<TB, VEC>(B, p.ldb, n0, p.N, (kt + 1) * BK16, p.K, t, rb);
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            bf8_t a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i)
                a[i] = *reinterpret_cast<const bf8_t*>(&As[cur][swz16(wm * 64 + i * 16 + l16, 4 * h + kg)]);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                b[j] = *reinterpret_cast<const bf8_t*>(&Bs[cur][swz16(wn * 64 + j * 16 + l16, 4 * h + kg)]);
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        if (more) {
            store16<!TA>(As[cur ^ 1], t, ra);
            store16<TB>(Bs[cur ^ 1], t, rb);
        }
        __syncthreads();
    }
    const double* __restrict__ C = p.C ? p.C + bz * p.sC : nullptr;
    double* __restrict__ D = p.Df ? nullptr : p.D + bz * p.sD;
    float* __restrict__ Df = p.Df ? p.Df + bz * p.sD : nullptr;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int col = n0 + wn * 64 + j * 16 + l16;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm * 64 + i * 16 + 4 * kg + r;
                if (row < p.M && col < p.N) {
                    double v = p.alpha * (double)acc[i][j][r];
                    if (Df) {
                        Df[(long)row * p.ldd + col] = (float)v;
                    } else {
                        if (C) v += p.beta * C[(long)row * p.ldc + col];
                        D[(long)row * p.ldd + col] = v;
                    }
                }
            }
        }
}

}  // namespace

void gemm_f64(const Gemm& g, hipStream_t s) { launch<double>(g, s); }

namespace {
// D[m][n] = alpha sum_b W[b][m][n] + beta C[m][n], the parts summed in order.
__global__ __launch_bounds__(256) void splitk_sum_kernel(const double* __restrict__ W, int parts, int M, int N,
                                                         double alpha, const double* C, long ldc, double beta,
                                                         double* D, long ldd) {
    const long n_all = (long)M * N, part = n_all;
    for (long e = blockIdx.x * 256L + threadIdx.x; e < n_all; e += (long)gridDim.x * 256) {
        double v = W[e];
        for (int b = 1; b < parts; ++b) v += W[b * part + e];
        const long m = e / N, n = e % N;
        v *= alpha;
        if (C) v += beta * C[m * ldc + n];
        D[m * ldd + n] = v;
    }
}
}  // namespace

int splitk_parts(int M, int N, int K, int slots) {
    const long tiles = (long)((M + BM - 1) / BM) * ((N + BN - 1) / BN);
    if (tiles * 2 > slots || K < 2048) return 1;
    int s = (int)std::min<long>(slots / tiles, K / 1024);
    while (s > 1 && K % (s * BK) != 0) --s;
    return std::max(s, 1);
}

// The K parts of g (no C, alpha 1) as one batched launch: part k to
// out + k part_stride (FP64) with row stride ldo.
template <typename T>
static void gemm_kparts(const Gemm& g, int parts, double* out, long ldo, long part_stride, hipStream_t s) {
    if (g.batch != 1 || g.Df) ITE_FAIL(ITE_EINVAL, "gemm K parts: single problems with an FP64 output only");
    if (parts < 1 || g.K % parts != 0) ITE_FAIL(ITE_EINVAL, "gemm K parts: K must split evenly");
    const int kp = g.K / parts;
    Gemm h = g;
    h.K = kp;
    h.batch = parts;
    h.sA = g.tA ? (long)kp * g.lda : kp;      // A stored K x M when transposed, else M x K
    h.sB = g.tB ? kp : (long)kp * g.ldb;      // B stored N x K when transposed, else K x N
    h.alpha = 1.0;
    h.beta = 0.0;
    h.C = nullptr;
    h.D = out;
    h.ldd = ldo;
    h.sD = part_stride;
    launch<T>(h, s);
}

template <typename T>
static void gemm_splitk(const Gemm& g, int parts, double* work, hipStream_t s) {
    if (parts <= 1) {
        launch<T>(g, s);
        return;
    }
    gemm_kparts<T>(g, parts, work, g.N, (long)g.M * g.N, s);
    const long n = (long)g.M * g.N;
    const int grid = (int)std::min<long>(4096, (n + 255) / 256);
    hipLaunchKernelGGL(splitk_sum_kernel, dim3(grid), dim3(256), 0, s, work, parts, g.M, g.N, g.alpha, g.C, g.ldc,
                       g.beta, g.D, g.ldd);
    HIP_CHECK(hipGetLastError());
}

void gemm_f64_splitk(const Gemm& g, int parts, double* work, hipStream_t s) { gemm_splitk<double>(g, parts, work, s); }
void gemm_f32_splitk(const Gemm& g, int parts, double* work, hipStream_t s) { gemm_splitk<float>(g, parts, work, s); }

size_t grouped_desc_bytes() { return sizeof(GroupDesc); }

// Host side of a grouped launch: the descriptor of problem g (its tiles
// start at tile_start) in the layout gemm_grouped_kernel reads.
void grouped_desc_fill(const Gemm& g, int bs, int tile_start, void* out) {
    GroupDesc d{};
    Params& p = d.p;
    p.M = g.M; p.N = g.N; p.K = g.K;
    p.alpha = g.alpha; p.beta = g.beta;
    p.A = g.A; p.lda = g.lda; p.sA = 0;
    p.B = g.B; p.ldb = g.ldb; p.sB = 0;
    p.C = g.C; p.ldc = g.ldc; p.sC = 0;
    p.D = g.D; p.ldd = g.ldd; p.sD = 0;
    p.Df = g.Df;
    p.mt = g.M > 0 ? (g.M + bs - 1) / bs : 0;
    p.nt = g.N > 0 ? (g.N + bs - 1) / bs : 0;
    d.tile_start = tile_start;
    std::memcpy(out, &d, sizeof(d));
}

int grouped_tiles(const Gemm& g, int bs) {
    if (g.M <= 0 || g.N <= 0) return 0;
    return ((g.M + bs - 1) / bs) * ((g.N + bs - 1) / bs);
}

void gemm_grouped_f32(const void* desc, const int* count, bool tA, bool tB, int grid, hipStream_t s) {
    const auto* d = static_cast<const GroupDesc*>(desc);
    if (!tA && !tB)
        hipLaunchKernelGGL((gemm_grouped_kernel<float, false, false, 128>), dim3(grid), dim3(NTHREADS), 0, s, d, count);
    else if (!tA && tB)
        hipLaunchKernelGGL((gemm_grouped_kernel<float, false, true, 128>), dim3(grid), dim3(NTHREADS), 0, s, d, count);
    else
        ITE_FAIL(ITE_EINVAL, "gemm_grouped_f32: transposed A is not supported");
    HIP_CHECK(hipGetLastError());
}

void gemm_grouped_f64(const void* desc, const int* count, bool tA, bool tB, int bs, int grid, hipStream_t s) {
    if (bs != 128 && bs != 64) ITE_FAIL(ITE_EINVAL, "gemm_grouped: tile must be 128 or 64");
    const auto* d = static_cast<const GroupDesc*>(desc);
#define ITE_GG(TA, TB, BS) \
    hipLaunchKernelGGL((gemm_grouped_kernel<double, TA, TB, BS>), dim3(grid), dim3(NTHREADS), 0, s, d, count)
    if (bs == 128) {
        if (!tA && !tB) ITE_GG(false, false, 128);
        else if (!tA && tB) ITE_GG(false, true, 128);
        else if (tA && !tB) ITE_GG(true, false, 128);
        else ITE_GG(true, true, 128);
    } else {
        if (!tA && !tB) ITE_GG(false, false, 64);
        else if (!tA && tB) ITE_GG(false, true, 64);
        else if (tA && !tB) ITE_GG(true, false, 64);
        else ITE_GG(true, true, 64);
    }
#undef ITE_GG
    HIP_CHECK(hipGetLastError());
}
void gemm_f32(const Gemm& g, hipStream_t s) { launch<float>(g, s); }

void gemm_bf16(const Gemm& g, hipStream_t s) {
    if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return;
    Params p;
    p.M = g.M; p.N = g.N; p.K = g.K;
    p.alpha = g.alpha; p.beta = g.beta;
    p.A = g.A; p.lda = g.lda; p.sA = g.sA;
    p.B = g.B; p.ldb = g.ldb; p.sB = g.sB;
    p.C = g.C; p.ldc = g.ldc; p.sC = g.sC;
    p.D = g.D; p.ldd = g.ldd; p.sD = g.sD;
    p.Df = g.Df;
    if (g.Df && g.C) ITE_FAIL(ITE_EINVAL, "gemm: an FP32 output takes no C");
    p.mt = (g.M + BM - 1) / BM;
    p.nt = (g.N + BN - 1) / BN;
    dim3 grid(p.mt * p.nt, 1, g.batch);
    const bool v = vec16(g, sizeof(uint16_t));
#define ITE_GB(TA, TB)                                                                               \
    if (v) hipLaunchKernelGGL((gemm_bf16_kernel<TA, TB, true>), grid, dim3(NTHREADS), 0, s, p);      \
    else hipLaunchKernelGGL((gemm_bf16_kernel<TA, TB, false>), grid, dim3(NTHREADS), 0, s, p)
    if (!g.tA && !g.tB) { ITE_GB(false, false); }
    else if (!g.tA && g.tB) { ITE_GB(false, true); }
    else if (g.tA && !g.tB) { ITE_GB(true, false); }
    else { ITE_GB(true, true); }
#undef ITE_GB
    HIP_CHECK(hipGetLastError());
}

void mfma_probe_f64(double* out, hipStream_t s) {
    hipLaunchKernelGGL(mfma_probe_kernel, dim3(1), dim3(64), 0, s, out);
    HIP_CHECK(hipGetLastError());
}

}  // namespace ite
