// Learned initializer: a small convolutional network that regresses lens
// parameters (and their log-variances) from a 64x64 image, trained and run
// with hand-written BF16 matrix-core (MFMA) kernels with FP32 accumulation.
//
// Every dense contraction (convolution forward, data gradient, weight
// gradient; fully connected forward and backward) is one generic GEMM kernel
// C[M][N] = sum_k A(m, k) B(k, n) whose operand loads and epilogue are given
// by small "op" structs (implicit GEMM: no im2col buffer).  Tiles: 64 x 64
// outputs per 256-thread work-group, K in steps of 32 staged through LDS,
// each wave computing 32 x 32 with 2 x 2 v_mfma_f32_16x16x32_bf16.
// Activations and gradients between layers are bf16 (round to nearest even);
// master weights, biases, Adam moments and reductions are fp32/fp64.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "lens_cnn.h"
#include "lens_philox.h"

namespace lens {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ __bf16 to_bf16(float x) { return (__bf16)x; }   // RNE
__device__ __forceinline__ float from_bf16(__bf16 x) { return (float)x; }
__device__ __forceinline__ bf16x8 zero8() {
    bf16x8 z;
#pragma unroll
    for (int i = 0; i < 8; ++i) z[i] = (__bf16)0.0f;
    return z;
}

__device__ __forceinline__ bf16x8 ld8(const __bf16* p) { return *reinterpret_cast<const bf16x8*>(p); }
// v where the layer input was positive, +0 elsewhere (the ReLU's data gradient)
__device__ __forceinline__ bf16x8 relu_mask8(bf16x8 v, bf16x8 prev) {
    bf16x8 r;
#pragma unroll
    for (int e = 0; e < 8; ++e) r[e] = from_bf16(prev[e]) > 0.0f ? v[e] : to_bf16(0.0f);
    return r;
}

// ---------------------------------------------------------------------------
// Generic BF16 MFMA GEMM.  Each operand is read either along K (row-major
// A[m][k], column-major B[k][n]: 8 consecutive k per 16-byte load) or, in
// "K-major" mode, along M (resp. N): 8 consecutive m at one k, transposed
// into the LDS tile as they are stored.  Op provides, per operand:
//   A along K: bf16x8 loadA(int m, int k, int kend)  -> A(m, k..k+7)
//   A K-major: bf16x8 loadAT(int k, int m)           -> A(m..m+7, k)
//   B along K: bf16x8 loadB(int k, int n, int kend)  -> B(k..k+7, n)
//   B K-major: bf16x8 loadBT(int k, int n)           -> B(k, n..n+7)
// (zero outside the matrix; K-major loads are called only for k < kend),
// constexpr bool A_KMAJOR, B_KMAJOR, and void store(int m, int n, float v,
// int split).
// ---------------------------------------------------------------------------
constexpr int GT = 64;    // output tile (M and N)
constexpr int GK = 64;    // K per stage (two MFMA K-steps of 32)
constexpr int LDSK = 72;  // padded LDS row (bf16)

// Precomputed gathers (ops with CTX_A / CTX_B).  An A row m (along K) is a
// base offset into the op's source and a mask of the taps that stay inside
// the image, both fixed across K stages; a K chunk is a tap bit and an
// offset, the same for every row of a thread:
//   GatherCtx a_row(int m), int a_koff(int k, int& bit), const __bf16* a_src()
//   A(m, k..k+7) = (mask >> bit) & 1 ? a_src()[base + koff ..] : 0.
// A K-major B (weight gradient: k = output position, n = (tap, ci)) has a
// row part per group of 8 n and a position part per k:
//   WRow b_row(int n), WPos b_pos(int k), bf16x8 b_load(WRow, WPos).
struct GatherCtx {
    int base;
    uint32_t mask;
};
struct WRow {
    int off, dy, dx;   // element offset and tap displacement; dy < -8: outside B
};
struct WPos {
    int base, iy, ix;
};

// XCD-aware tile order.  The dispatcher hands work-group L (in x, y, z order)
// to XCD L mod 8, and each XCD has its own L2, so neighbouring tiles that
// read the same operand rows (the N tiles of one K split, adjacent M tiles
// with shared halo rows) would each fetch them from HBM.  The logical tile
// of work-group L is taken so that every XCD runs one contiguous range of
// logical tiles (x fastest, then y, then z): a bijection of the grid.  Used
// where several N tiles or K splits exist (the weight gradients).
struct TileIdx {
    int x, y, z;
};
constexpr int N_XCD = 8;

__device__ __forceinline__ TileIdx xcd_tile() {
    const int gx = gridDim.x, gy = gridDim.y;
    // one N tile and no K split: dispatch order (measured faster there)
    if (gy == 1 && gridDim.z == 1) return TileIdx{(int)blockIdx.x, 0, 0};
    const int n = gx * gy * gridDim.z;
    const int L = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    const int per = n / N_XCD, rem = n % N_XCD;
    const int x = L % N_XCD, i = L / N_XCD;
    const int g = x * per + min(x, rem) + i;   // XCD x: logical tiles [x per + min(x, rem), ...)
    return TileIdx{g % gx, (g / gx) % gy, g / (gx * gy)};
}

// Ops that run several GEMMs of one output shape in one launch (the four
// input-parity classes of a stride-2 data gradient) define CLASSES = true,
// set_class(c) and class_k() (the K extent of class c); the launch has
// gridDim.z = number of classes and no K split.
template <class Op, class = void>
struct has_classes {
    static constexpr bool value = false;
};
template <class Op>
struct has_classes<Op, decltype((void)Op::CLASSES)> {
    static constexpr bool value = Op::CLASSES;
};

// Tile order of a class launch: the classes of one output tile are read
// from the same operand rows, so they run back to back on one XCD (one L2).
// Work-group L goes to XCD L mod 8 as its (L / 8)-th group there; in each
// run of 32 work-groups the four classes of tile i / 4 * 8 + L mod 8 follow
// each other on that XCD.  The remainder (fewer than 32) is in dispatch order.
__device__ __forceinline__ TileIdx class_tile() {
    const int gx = gridDim.x, nc = gridDim.z;
    const int L = blockIdx.x + gx * (blockIdx.y + gridDim.y * blockIdx.z);
    const int n = gx * gridDim.y * nc, full = n / (N_XCD * nc) * (N_XCD * nc);
    int cls, t;
    if (L < full) {
        const int x = L % N_XCD, i = L / N_XCD;
        cls = i % nc;
        t = (i / nc) * N_XCD + x;
    } else {
        cls = (L - full) % nc;
        t = full / nc + (L - full) / nc;
    }
    return TileIdx{t % gx, t / gx, cls};
}

// Loads of one stage into registers: along K, thread t covers row t/4 at
// k offsets 8 (t%4) and 32 + 8 (t%4); K-major, k t%64 at rows 8 (t/64) and
// 32 + 8 (t/64).
template <class Op>
struct StageRegs {
    bf16x8 a[2], b[2];
    GatherCtx actx;   // CTX_A: this thread's A row
    WRow brow[2];     // CTX_B: this thread's B row groups
};

template <class Op>
__device__ __forceinline__ void load_stage(const Op& op, StageRegs<Op>& r, int m0, int n0, int k0, int kend, int M,
                                           int N) {
    const int t = threadIdx.x;
    const int lr = t >> 2, lk = (t & 3) * 8;
    const int tk = t & 63, tr = (t >> 6) * 8;
    WPos bp{};
    if constexpr (Op::CTX_B) {
        if (k0 + tk < kend) bp = op.b_pos(k0 + tk);
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        if constexpr (Op::A_KMAJOR) {
            r.a[h] = (k0 + tk < kend) ? op.loadAT(k0 + tk, m0 + tr + 32 * h) : zero8();
        } else if constexpr (Op::CTX_A) {
            const int k = k0 + lk + 32 * h;
            int bit = 0;
            const int off = k < kend ? op.a_koff(k, bit) : 0;
            r.a[h] = (k < kend && ((r.actx.mask >> bit) & 1u)) ? ld8(op.a_src() + r.actx.base + off) : zero8();
        } else {
            r.a[h] = (m0 + lr < M) ? op.loadA(m0 + lr, k0 + lk + 32 * h, kend) : zero8();
        }
        if constexpr (Op::CTX_B)
            r.b[h] = (k0 + tk < kend) ? op.b_load(r.brow[h], bp) : zero8();
        else if constexpr (Op::B_KMAJOR)
            r.b[h] = (k0 + tk < kend) ? op.loadBT(k0 + tk, n0 + tr + 32 * h) : zero8();
        else
            r.b[h] = (n0 + lr < N) ? op.loadB(k0 + lk + 32 * h, n0 + lr, kend) : zero8();
    }
}

// The row parts of a thread's gathers (fixed for the whole K range).
template <class Op>
__device__ __forceinline__ void init_stage_ctx(const Op& op, StageRegs<Op>& r, int m0, int n0, int M, int N) {
    const int t = threadIdx.x;
    if constexpr (Op::CTX_A && !Op::A_KMAJOR) r.actx = (m0 + (t >> 2) < M) ? op.a_row(m0 + (t >> 2)) : GatherCtx{0, 0u};
    if constexpr (Op::CTX_B) {
#pragma unroll
        for (int h = 0; h < 2; ++h) r.brow[h] = op.b_row(n0 + (t >> 6) * 8 + 32 * h);
    }
}

template <class Op>
__device__ __forceinline__ void store_stage(const StageRegs<Op>& r, __bf16 (*As)[LDSK], __bf16 (*Bs)[LDSK]) {
    const int t = threadIdx.x;
    const int lr = t >> 2, lk = (t & 3) * 8;
    const int tk = t & 63, tr = (t >> 6) * 8;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        if constexpr (Op::A_KMAJOR) {
#pragma unroll
            for (int i = 0; i < 8; ++i) As[tr + 32 * h + i][tk] = r.a[h][i];
        } else {
            *reinterpret_cast<bf16x8*>(&As[lr][lk + 32 * h]) = r.a[h];
        }
        if constexpr (Op::B_KMAJOR) {
#pragma unroll
            for (int i = 0; i < 8; ++i) Bs[tr + 32 * h + i][tk] = r.b[h][i];
        } else {
            *reinterpret_cast<bf16x8*>(&Bs[lr][lk + 32 * h]) = r.b[h];
        }
    }
}

// C[M][N] over K in [blockIdx.z * k_per_split, ...): 64 x 64 tile per
// 256-thread work-group, each wave 32 x 32 (2 x 2 MFMA 16x16x32 tiles).  The
// next stage's global loads are issued before the current stage's MFMAs.
template <class Op>
__global__ __launch_bounds__(256) void k_gemm(Op op, int M, int N, int K, int k_per_split) {
    __shared__ __attribute__((aligned(16))) __bf16 As[GT][LDSK];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[GT][LDSK];
    const TileIdx tb = xcd_tile();
    const int m0 = tb.x * GT, n0 = tb.y * GT;
    const int kbeg = tb.z * k_per_split;
    const int kend = min(K, kbeg + k_per_split);
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wm = w >> 1, wn = w & 1;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    StageRegs<Op> r;
    init_stage_ctx(op, r, m0, n0, M, N);
    if (kbeg < kend) load_stage(op, r, m0, n0, kbeg, kend, M, N);
    for (int k0 = kbeg; k0 < kend; k0 += GK) {
        __syncthreads();
        store_stage(r, As, Bs);
        __syncthreads();
        if (k0 + GK < kend) load_stage(op, r, m0, n0, k0 + GK, kend, M, N);
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const bf16x8 a =
                    *reinterpret_cast<const bf16x8*>(&As[32 * wm + 16 * i + (lane & 15)][32 * kk + 8 * (lane >> 4)]);
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const bf16x8 b = *reinterpret_cast<const bf16x8*>(
                        &Bs[32 * wn + 16 * j + (lane & 15)][32 * kk + 8 * (lane >> 4)]);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[i][j], 0, 0, 0);
                }
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int m = m0 + 32 * wm + 16 * i + 4 * (lane >> 4) + q;
                const int n = n0 + 32 * wn + 16 * j + (lane & 15);
                if (m < M && n < N) op.store(m, n, acc[i][j][q], tb.z);
            }
}

// Tall tile for GEMMs with large M (convolution forward and data gradient):
// 128 x 64 outputs per work-group, wave w computing rows 32 w .. 32 w + 31 of
// all 64 columns (2 x 4 MFMA tiles), so each B stage feeds twice the rows.
constexpr int GT2 = 128;

template <class Op>
struct StageRegs2 {
    bf16x8 a[4], b[2];
    GatherCtx actx;   // CTX_A: this thread's A row
};

template <class Op>
__device__ __forceinline__ void load_stage2(const Op& op, StageRegs2<Op>& r, int m0, int n0, int k0, int kend, int M,
                                            int N) {
    const int t = threadIdx.x;
    const int ar = t >> 1, ak = (t & 1) * 32;        // A along K: row t/2, k 32 (t%2) + 8 h
    const int br = t >> 2, bk = (t & 3) * 8;         // B along K: row t/4, k 8 (t%4) + 32 h
    const int tk = t & 63, tr = (t >> 6) * 8;        // K-major: k t%64, rows 8 (t/64) + 32 h
#pragma unroll
    for (int h = 0; h < 4; ++h) {
        if constexpr (Op::A_KMAJOR) {
            r.a[h] = (k0 + tk < kend) ? op.loadAT(k0 + tk, m0 + tr + 32 * h) : zero8();
        } else if constexpr (Op::CTX_A) {
            const int k = k0 + ak + 8 * h;
            int bit = 0;
            const int off = k < kend ? op.a_koff(k, bit) : 0;
            r.a[h] = (k < kend && ((r.actx.mask >> bit) & 1u)) ? ld8(op.a_src() + r.actx.base + off) : zero8();
        } else {
            r.a[h] = (m0 + ar < M) ? op.loadA(m0 + ar, k0 + ak + 8 * h, kend) : zero8();
        }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        if constexpr (Op::B_KMAJOR)
            r.b[h] = (k0 + tk < kend) ? op.loadBT(k0 + tk, n0 + tr + 32 * h) : zero8();
        else
            r.b[h] = (n0 + br < N) ? op.loadB(k0 + bk + 32 * h, n0 + br, kend) : zero8();
    }
}

template <class Op>
__device__ __forceinline__ void store_stage2(const StageRegs2<Op>& r, __bf16 (*As)[LDSK], __bf16 (*Bs)[LDSK]) {
    const int t = threadIdx.x;
    const int ar = t >> 1, ak = (t & 1) * 32;
    const int br = t >> 2, bk = (t & 3) * 8;
    const int tk = t & 63, tr = (t >> 6) * 8;
#pragma unroll
    for (int h = 0; h < 4; ++h) {
        if constexpr (Op::A_KMAJOR) {
#pragma unroll
            for (int i = 0; i < 8; ++i) As[tr + 32 * h + i][tk] = r.a[h][i];
        } else {
            *reinterpret_cast<bf16x8*>(&As[ar][ak + 8 * h]) = r.a[h];
        }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        if constexpr (Op::B_KMAJOR) {
#pragma unroll
            for (int i = 0; i < 8; ++i) Bs[tr + 32 * h + i][tk] = r.b[h][i];
        } else {
            *reinterpret_cast<bf16x8*>(&Bs[br][bk + 32 * h]) = r.b[h];
        }
    }
}

// Epilogue of ops with STORE8 (bf16 row-major outputs, N a multiple of 8):
// the tile is converted (op.pre: bias, activation) and staged as bf16 in
// LDS, then written 8 columns (16 bytes) per thread with op.store8.
// C points at TM x (TN + 8) bf16 of LDS that no wave reads any more.
template <class Op, int TM, int TN>
__device__ __forceinline__ void store_tile8(const Op& op, __bf16* C, int m0, int n0, int M, int N) {
    constexpr int CW = TN + 8;
#pragma unroll
    for (int h = 0; h < TM * TN / 2048; ++h) {
        const int c = threadIdx.x + 256 * h;
        const int ml = c / (TN / 8), nl = (c % (TN / 8)) * 8;
        if (m0 + ml < M && n0 + nl < N)
            op.store8(m0 + ml, n0 + nl, *reinterpret_cast<const bf16x8*>(&C[ml * CW + nl]));
    }
}

template <class Op>
__global__ __launch_bounds__(256) void k_gemm_tall(Op op, int M, int N, int K, int k_per_split) {
    __shared__ __attribute__((aligned(16))) __bf16 smem[(GT2 + GT) * LDSK];
    __bf16 (*As)[LDSK] = reinterpret_cast<__bf16 (*)[LDSK]>(smem);
    __bf16 (*Bs)[LDSK] = reinterpret_cast<__bf16 (*)[LDSK]>(smem + GT2 * LDSK);
    const TileIdx tb = xcd_tile();
    const int m0 = tb.x * GT2, n0 = tb.y * GT;
    const int kbeg = tb.z * k_per_split;
    const int kend = min(K, kbeg + k_per_split);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    f32x4 acc[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    StageRegs2<Op> r;
    if constexpr (Op::CTX_A && !Op::A_KMAJOR) {
        const int row = m0 + (threadIdx.x >> 1);
        r.actx = row < M ? op.a_row(row) : GatherCtx{0, 0u};
    }
    if (kbeg < kend) load_stage2(op, r, m0, n0, kbeg, kend, M, N);
    for (int k0 = kbeg; k0 < kend; k0 += GK) {
        __syncthreads();
        store_stage2(r, As, Bs);
        __syncthreads();
        if (k0 + GK < kend) load_stage2(op, r, m0, n0, k0 + GK, kend, M, N);
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
            bf16x8 bv[4];
#pragma unroll
            for (int j = 0; j < 4; ++j)
                bv[j] = *reinterpret_cast<const bf16x8*>(&Bs[16 * j + (lane & 15)][32 * kk + 8 * (lane >> 4)]);
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const bf16x8 a =
                    *reinterpret_cast<const bf16x8*>(&As[32 * w + 16 * i + (lane & 15)][32 * kk + 8 * (lane >> 4)]);
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bv[j], acc[i][j], 0, 0, 0);
            }
        }
    }
    if constexpr (Op::STORE8) {
        static_assert(GT2 * (GT + 8) <= (GT2 + GT) * LDSK, "staged tile fits the operand tiles");
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int ml = 32 * w + 16 * i + 4 * (lane >> 4) + q, nl = 16 * j + (lane & 15);
                    smem[ml * (GT + 8) + nl] = n0 + nl < N ? op.pre(m0 + ml, n0 + nl, acc[i][j][q]) : to_bf16(0.0f);
                }
        __syncthreads();
        store_tile8<Op, GT2, GT>(op, smem, m0, n0, M, N);
    } else {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int m = m0 + 32 * w + 16 * i + 4 * (lane >> 4) + q;
                    const int n = n0 + 16 * j + (lane & 15);
                    if (m < M && n < N) op.store(m, n, acc[i][j][q], tb.z);
                }
    }
}

// Large tiles: 4 waves arranged WM x WN, each computing 64 x 64 outputs
// (4 x 4 MFMA 16x16x32 tiles): 128 x 128 (2 x 2), 256 x 64 (4 x 1) or
// 64 x 256 (1 x 4) per work-group; or 64 x 32 each (4 x 2 tiles, JT = 2)
// for 256 x 32.  Per MFMA a wave reads half a fragment
// from LDS (8 fragments per 16 MFMAs) against three quarters with the 32-row
// wave tiles above.
template <class Op, int R>
struct WideRegs {
    bf16x8 v[R / 32];   // R rows x 64 k of one operand, 2 R / 64 chunks of 8 per thread
};

// Gathered rows of one operand of the wide kernels: along K the thread's
// rows are r0 + t/8 + 32 h (A rows, GatherCtx); K-major its row groups are
// r0 + 8 (t/64 + 4 h) (B row groups, WRow).
template <int R>
struct WideCtx {
    GatherCtx a[R / 32];
    WRow b[R / 32];
};

template <int R, class Op>
__device__ __forceinline__ void wide_ctx_a(const Op& op, WideCtx<R>& c, int r0, int rows) {
    const int t = threadIdx.x;
#pragma unroll
    for (int h = 0; h < R / 32; ++h) {
        const int row = r0 + (t >> 3) + 32 * h;
        c.a[h] = row < rows ? op.a_row(row) : GatherCtx{0, 0u};
    }
}

template <int R, class Op>
__device__ __forceinline__ void wide_ctx_b(const Op& op, WideCtx<R>& c, int r0) {
    const int t = threadIdx.x;
#pragma unroll
    for (int h = 0; h < R / 32; ++h) c.b[h] = op.b_row(r0 + 8 * ((t >> 6) + 4 * h));
}

// rows x 64 k of A along K through the row contexts.
template <int R, class Op>
__device__ __forceinline__ void wide_load_actx(const Op& op, WideRegs<void, R>& r, const WideCtx<R>& c, int k0,
                                               int kend) {
    const int k = k0 + (threadIdx.x & 7) * 8;
    int bit = 0;
    const int off = k < kend ? op.a_koff(k, bit) : 0;
    const __bf16* src = op.a_src();
#pragma unroll
    for (int h = 0; h < R / 32; ++h)
        r.v[h] = (k < kend && ((c.a[h].mask >> bit) & 1u)) ? ld8(src + c.a[h].base + off) : zero8();
}

// 64 k x rows of a K-major B through the row-group contexts.
template <int R, class Op>
__device__ __forceinline__ void wide_load_bctx(const Op& op, WideRegs<void, R>& r, const WideCtx<R>& c, int k0,
                                               int kend) {
    const int k = k0 + (threadIdx.x & 63);
    if (k >= kend) {
#pragma unroll
        for (int h = 0; h < R / 32; ++h) r.v[h] = zero8();
        return;
    }
    const WPos p = op.b_pos(k);
#pragma unroll
    for (int h = 0; h < R / 32; ++h) r.v[h] = op.b_load(c.b[h], p);
}

// rows x 64 k of one operand into registers: along K, chunk c = t + 256 h covers
// row c / 8 at k 8 (c % 8); K-major, chunk c covers k c % 64 at rows 8 (c / 64).
template <bool KMAJOR, int R, class F, class FT>
__device__ __forceinline__ void wide_load(WideRegs<void, R>& r, int r0, int k0, int kend, int rows, F&& ld, FT&& ldt) {
    const int t = threadIdx.x;
#pragma unroll
    for (int h = 0; h < R / 32; ++h) {
        const int c = t + 256 * h;
        if constexpr (KMAJOR) {
            const int k = c & 63, rg = c >> 6;
            r.v[h] = (k0 + k < kend) ? ldt(k0 + k, r0 + 8 * rg) : zero8();
        } else {
            const int row = c >> 3, kc = (c & 7) * 8;
            r.v[h] = (r0 + row < rows) ? ld(r0 + row, k0 + kc, kend) : zero8();
        }
    }
}

template <bool KMAJOR, int R>
__device__ __forceinline__ void wide_store(const WideRegs<void, R>& r, __bf16 (*S)[LDSK]) {
    const int t = threadIdx.x;
#pragma unroll
    for (int h = 0; h < R / 32; ++h) {
        const int c = t + 256 * h;
        if constexpr (KMAJOR) {
            const int k = c & 63, rg = c >> 6;
#pragma unroll
            for (int i = 0; i < 8; ++i) S[8 * rg + i][k] = r.v[h][i];
        } else {
            const int row = c >> 3, kc = (c & 7) * 8;
            *reinterpret_cast<bf16x8*>(&S[row][kc]) = r.v[h];
        }
    }
}

template <class Op, int WM, int WN, int JT = 4>
__global__ __launch_bounds__(256) void k_gemm_wide(Op op0, int M, int N, int K, int k_per_split) {
    constexpr int TM = 64 * WM, TN = 16 * JT * WN;   // each wave: 64 x 16 JT outputs
    constexpr bool CLS = has_classes<Op>::value;
    __shared__ __attribute__((aligned(16))) __bf16 smem[(TM + TN) * LDSK];
    __bf16 (*As)[LDSK] = reinterpret_cast<__bf16 (*)[LDSK]>(smem);
    __bf16 (*Bs)[LDSK] = reinterpret_cast<__bf16 (*)[LDSK]>(smem + TM * LDSK);
    const TileIdx tb = CLS ? class_tile() : xcd_tile();
    Op op = op0;
    if constexpr (CLS) {
        op.set_class(tb.z);
        K = op.class_k();
        k_per_split = K;
    }
    const int m0 = tb.x * TM, n0 = tb.y * TN;
    const int kbeg = CLS ? 0 : tb.z * k_per_split;
    const int kend = min(K, kbeg + k_per_split);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wm = w / WN, wn = w % WN;
    f32x4 acc[4][JT];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < JT; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    auto la = [&](int m, int k, int ke) {
        if constexpr (!Op::A_KMAJOR) return op.loadA(m, k, ke);
        else return zero8();
    };
    auto lat = [&](int k, int m) {
        if constexpr (Op::A_KMAJOR) return op.loadAT(k, m);
        else return zero8();
    };
    auto lb = [&](int n, int k, int ke) {
        if constexpr (!Op::B_KMAJOR) return op.loadB(k, n, ke);
        else return zero8();
    };
    auto lbt = [&](int k, int n) {
        if constexpr (Op::B_KMAJOR) return op.loadBT(k, n);
        else return zero8();
    };
    WideRegs<void, TM> ra;
    WideRegs<void, TN> rb;
    WideCtx<TM> ca;
    WideCtx<TN> cb;
    if constexpr (Op::CTX_A && !Op::A_KMAJOR) wide_ctx_a(op, ca, m0, M);
    if constexpr (Op::CTX_B) wide_ctx_b(op, cb, n0);
    auto load_a = [&](int k0) {
        if constexpr (Op::CTX_A && !Op::A_KMAJOR) wide_load_actx(op, ra, ca, k0, kend);
        else wide_load<Op::A_KMAJOR, TM>(ra, m0, k0, kend, M, la, lat);
    };
    auto load_b = [&](int k0) {
        if constexpr (Op::CTX_B) wide_load_bctx(op, rb, cb, k0, kend);
        else wide_load<Op::B_KMAJOR, TN>(rb, n0, k0, kend, N, lb, lbt);
    };
    if (kbeg < kend) {
        load_a(kbeg);
        load_b(kbeg);
    }
    for (int k0 = kbeg; k0 < kend; k0 += GK) {
        __syncthreads();
        wide_store<Op::A_KMAJOR, TM>(ra, As);
        wide_store<Op::B_KMAJOR, TN>(rb, Bs);
        __syncthreads();
        if (k0 + GK < kend) {
            load_a(k0 + GK);
            load_b(k0 + GK);
        }
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
            bf16x8 av[4], bv[JT];
#pragma unroll
            for (int i = 0; i < 4; ++i)
                av[i] = *reinterpret_cast<const bf16x8*>(&As[64 * wm + 16 * i + (lane & 15)][32 * kk + 8 * (lane >> 4)]);
#pragma unroll
            for (int j = 0; j < JT; ++j)
                bv[j] = *reinterpret_cast<const bf16x8*>(
                    &Bs[16 * JT * wn + 16 * j + (lane & 15)][32 * kk + 8 * (lane >> 4)]);
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < JT; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bv[j], acc[i][j], 0, 0, 0);
        }
    }
    if constexpr (Op::STORE8) {
        static_assert(TM * (TN + 8) <= (TM + TN) * LDSK, "staged tile fits the operand tiles");
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < JT; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int ml = 64 * wm + 16 * i + 4 * (lane >> 4) + q, nl = 16 * JT * wn + 16 * j + (lane & 15);
                    smem[ml * (TN + 8) + nl] = n0 + nl < N ? op.pre(m0 + ml, n0 + nl, acc[i][j][q]) : to_bf16(0.0f);
                }
        __syncthreads();
        store_tile8<Op, TM, TN>(op, smem, m0, n0, M, N);
    } else {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < JT; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int m = m0 + 64 * wm + 16 * i + 4 * (lane >> 4) + q;
                    const int n = n0 + 16 * JT * wn + 16 * j + (lane & 15);
                    if (m < M && n < N) op.store(m, n, acc[i][j][q], tb.z);
                }
    }
}

// ---------------------------------------------------------------------------
// Operand maps.  NHWC activations; conv weights W[co][ky][kx][ci] (row co of
// length 9*Cin); fully connected W[out][in].  Every spatial size and channel
// count of the network is a power of two: index arithmetic uses shifts.
// ---------------------------------------------------------------------------
struct ConvShape {
    int B, H, W, Cin, Ho, Wo, Cout, stride;
    int lW, lWo, lCin, lCout;   // log2 of W, Wo, Cin, Cout
};

__host__ __device__ inline int ilog2(int v) {
    int l = 0;
    while ((1 << (l + 1)) <= v) ++l;
    return l;
}

inline ConvShape conv_shape(int B, int H, int Cin, int Ho, int Cout, int stride) {
    return ConvShape{B, H, H, Cin, Ho, Ho, Cout, stride, ilog2(H), ilog2(Ho), ilog2(Cin), ilog2(Cout)};
}

__device__ __forceinline__ int div3(int tap) { return (tap * 11) >> 5; }   // tap in [0, 9)


// forward: out[b,y,x,co] = relu(sum in[b, s y + ky - 1, s x + kx - 1, ci] W[co,ky,kx,ci] + bias)
// A(m = (b, y, x), k = (tap, ci)) along K; B(k, n = co) = W[co][k] along K.
struct OpConvFwd {
    static constexpr bool A_KMAJOR = false, B_KMAJOR = false;
    ConvShape s;
    const __bf16* in;
    const __bf16* w;
    const float* bias;
    __bf16* out;
    static constexpr bool CTX_A = true, CTX_B = false;   // gathers need Cin >= 8
    __device__ GatherCtx a_row(int m) const {
        const int b = m >> (2 * s.lWo), r = m & ((1 << (2 * s.lWo)) - 1);
        const int iy0 = (r >> s.lWo) * s.stride - 1, ix0 = (r & (s.Wo - 1)) * s.stride - 1;
        uint32_t mask = 0;
#pragma unroll
        for (int ky = 0; ky < 3; ++ky)
#pragma unroll
            for (int kx = 0; kx < 3; ++kx)
                if (iy0 + ky >= 0 && iy0 + ky < s.H && ix0 + kx >= 0 && ix0 + kx < s.W) mask |= 1u << (3 * ky + kx);
        return GatherCtx{((b * s.H + iy0) * s.W + ix0) * s.Cin, mask};
    }
    __device__ int a_koff(int k, int& bit) const {
        const int tap = k >> s.lCin, ky = div3(tap);
        bit = tap;
        return (ky * s.W + (tap - 3 * ky)) * s.Cin + (k & (s.Cin - 1));
    }
    __device__ const __bf16* a_src() const { return in; }
    __device__ bf16x8 loadA(int m, int k, int kend) const {
        const int b = m >> (2 * s.lWo), r = m & ((1 << (2 * s.lWo)) - 1);
        const int y = r >> s.lWo, x = r & (s.Wo - 1);
        bf16x8 v = zero8();
        if (s.Cin >= 8) {
            if (k >= kend) return v;
            const int tap = k >> s.lCin, ci = k & (s.Cin - 1), ky = div3(tap);
            const int iy = y * s.stride + ky - 1, ix = x * s.stride + (tap - 3 * ky) - 1;
            if (iy < 0 || iy >= s.H || ix < 0 || ix >= s.W) return v;
            return ld8(in + ((((size_t)b << s.lW) + iy) << s.lW) * s.Cin + ((size_t)ix << s.lCin) + ci);
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {   // Cin = 1 (first layer): k is the tap
            const int tap = k + q;
            if (tap >= kend) break;
            const int ky = div3(tap);
            const int iy = y * s.stride + ky - 1, ix = x * s.stride + (tap - 3 * ky) - 1;
            if (iy >= 0 && iy < s.H && ix >= 0 && ix < s.W) v[q] = in[(((size_t)b << s.lW) + iy) * s.W + ix];
        }
        return v;
    }
    __device__ bf16x8 loadB(int k, int n, int kend) const {
        const int KK = 9 * s.Cin;
        if (s.Cin >= 8) return k < kend ? ld8(w + (size_t)n * KK + k) : zero8();
        bf16x8 v = zero8();
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (k + q < kend) v[q] = w[(size_t)n * KK + k + q];
        return v;
    }
    __device__ void store(int m, int n, float v, int) const {
        out[((size_t)m << s.lCout) + n] = to_bf16(fmaxf(v + bias[n], 0.0f));
    }
    static constexpr bool STORE8 = true;
    __device__ __bf16 pre(int, int n, float v) const { return to_bf16(fmaxf(v + bias[n], 0.0f)); }
    __device__ void store8(int m, int n, bf16x8 v) const {
        *reinterpret_cast<bf16x8*>(out + ((size_t)m << s.lCout) + n) = v;
    }
};

// data gradient: dX[b,iy,ix,ci] = sum dZ[b,y,x,co] W[co,ky,kx,ci] over iy = s y + ky - 1,
// times the ReLU mask of the layer input (prev > 0) -> dZ of the previous layer.
// A(m = (b, iy, ix), k = (tap, co)) = dZ[b, y, x, co] along K (Cout >= 8);
// B(k = (tap, co), n = ci) = W[co][tap][ci]: K-major.
struct OpConvDgrad {
    static constexpr bool A_KMAJOR = false, B_KMAJOR = true;
    ConvShape s;
    const __bf16* dz;     // [B][Ho][Wo][Cout]
    const __bf16* w;
    const __bf16* prev;   // layer input (the previous layer's ReLU output)
    __bf16* dprev;        // [B][H][W][Cin]
    // gathers: stride 1 only (stride-2 layers use OpConvDgradS2)
    static constexpr bool CTX_A = true, CTX_B = false;
    __device__ GatherCtx a_row(int m) const {
        const int b = m >> (2 * s.lW), r = m & ((1 << (2 * s.lW)) - 1);
        const int iy = r >> s.lW, ix = r & (s.W - 1);
        uint32_t mask = 0;
#pragma unroll
        for (int ky = 0; ky < 3; ++ky)
#pragma unroll
            for (int kx = 0; kx < 3; ++kx)
                if (iy + 1 - ky >= 0 && iy + 1 - ky < s.Ho && ix + 1 - kx >= 0 && ix + 1 - kx < s.Wo)
                    mask |= 1u << (3 * ky + kx);
        return GatherCtx{((b * s.Ho + iy + 1) * s.Wo + ix + 1) * s.Cout, mask};
    }
    __device__ int a_koff(int k, int& bit) const {
        const int tap = k >> s.lCout, ky = div3(tap);
        bit = tap;
        return (k & (s.Cout - 1)) - (ky * s.Wo + (tap - 3 * ky)) * s.Cout;
    }
    __device__ const __bf16* a_src() const { return dz; }
    __device__ bf16x8 loadA(int m, int k, int kend) const {
        const int b = m >> (2 * s.lW), r = m & ((1 << (2 * s.lW)) - 1);
        const int iy = r >> s.lW, ix = r & (s.W - 1);
        if (k >= kend) return zero8();
        const int tap = k >> s.lCout, co = k & (s.Cout - 1), ky = div3(tap);
        const int ty = iy + 1 - ky, tx = ix + 1 - (tap - 3 * ky);
        if (ty < 0 || tx < 0 || (ty & (s.stride - 1)) || (tx & (s.stride - 1))) return zero8();
        const int y = ty >> (s.stride - 1), x = tx >> (s.stride - 1);   // stride 1 or 2
        if (y >= s.Ho || x >= s.Wo) return zero8();
        return ld8(dz + ((((size_t)b << s.lWo) + y) << s.lWo) * s.Cout + ((size_t)x << s.lCout) + co);
    }
    __device__ bf16x8 loadBT(int k, int n) const {
        if (n >= s.Cin) return zero8();
        const int tap = k >> s.lCout, co = k & (s.Cout - 1);
        return ld8(w + (size_t)co * 9 * s.Cin + ((size_t)tap << s.lCin) + n);
    }
    __device__ void store(int m, int n, float v, int) const {
        const size_t q = ((size_t)m << s.lCin) + n;
        dprev[q] = to_bf16(from_bf16(prev[q]) > 0.0f ? v : 0.0f);
    }
    static constexpr bool STORE8 = true;
    __device__ __bf16 pre(int, int, float v) const { return to_bf16(v); }
    __device__ void store8(int m, int n, bf16x8 v) const {
        const size_t q = ((size_t)m << s.lCin) + n;
        *reinterpret_cast<bf16x8*>(dprev + q) = relu_mask8(v, ld8(prev + q));
    }
};

// data gradient of a stride-2 layer, one input-parity class (py, px) per
// GEMM: input pixel (2 y' + py, 2 x' + px) receives output (y, x) only through
// taps ky = 1 (py = 0) or ky in {0, 2} (py = 1), likewise kx, so each class
// sums over 1, 2, 2 or 4 taps instead of 9 (the other taps meet no output).
// A(m = (b, y', x'), k = (t, co)) = dZ[b, y, x, co] along K; B(k, n = ci) =
// W[co][tap][ci]: K-major.  Output and ReLU mask as OpConvDgrad.
struct OpConvDgradS2 {
    static constexpr bool A_KMAJOR = false, B_KMAJOR = true;
    ConvShape s;   // stride 2: H = 2 Ho
    int py, px;
    const __bf16* dz;
    const __bf16* w;
    const __bf16* prev;
    __bf16* dprev;
    __device__ __forceinline__ void tap(int t, int& ky, int& kx) const {
        const int ntx = px ? 2 : 1;
        const int ty = px ? (t >> 1) : t, tx = px ? (t & 1) : 0;
        ky = py ? 2 * ty : 1;
        kx = px ? 2 * tx : 1;
        (void)ntx;
    }
    static constexpr bool CTX_A = true, CTX_B = false;
    // tap t reads dZ at (yq + dy, xq + dx), dy = (py + 1 - ky) / 2 in {0, 1}
    __device__ GatherCtx a_row(int m) const {
        const int b = m >> (2 * s.lWo), r = m & ((1 << (2 * s.lWo)) - 1);
        const int yq = r >> s.lWo, xq = r & (s.Wo - 1);
        const int ntap = (py ? 2 : 1) * (px ? 2 : 1);
        uint32_t mask = 0;
        for (int t = 0; t < ntap; ++t) {
            int ky, kx;
            tap(t, ky, kx);
            if (yq + ((py + 1 - ky) >> 1) < s.Ho && xq + ((px + 1 - kx) >> 1) < s.Wo) mask |= 1u << t;
        }
        return GatherCtx{((b * s.Ho + yq) * s.Wo + xq) * s.Cout, mask};
    }
    __device__ int a_koff(int k, int& bit) const {
        const int t = k >> s.lCout;
        int ky, kx;
        tap(t, ky, kx);
        bit = t;
        return (((py + 1 - ky) >> 1) * s.Wo + ((px + 1 - kx) >> 1)) * s.Cout + (k & (s.Cout - 1));
    }
    __device__ const __bf16* a_src() const { return dz; }
    __device__ bf16x8 loadA(int m, int k, int kend) const {
        if (k >= kend) return zero8();
        const int b = m >> (2 * s.lWo), r = m & ((1 << (2 * s.lWo)) - 1);
        const int yq = r >> s.lWo, xq = r & (s.Wo - 1);
        const int t = k >> s.lCout, co = k & (s.Cout - 1);
        int ky, kx;
        tap(t, ky, kx);
        const int y = yq + ((py + 1 - ky) >> 1), x = xq + ((px + 1 - kx) >> 1);
        if (y >= s.Ho || x >= s.Wo) return zero8();
        return ld8(dz + ((((size_t)b << s.lWo) + y) << s.lWo) * s.Cout + ((size_t)x << s.lCout) + co);
    }
    __device__ bf16x8 loadBT(int k, int n) const {
        if (n >= s.Cin) return zero8();
        const int t = k >> s.lCout, co = k & (s.Cout - 1);
        int ky, kx;
        tap(t, ky, kx);
        return ld8(w + (size_t)co * 9 * s.Cin + ((size_t)(3 * ky + kx) << s.lCin) + n);
    }
    __device__ void store(int m, int n, float v, int) const {
        const int b = m >> (2 * s.lWo), r = m & ((1 << (2 * s.lWo)) - 1);
        const int yq = r >> s.lWo, xq = r & (s.Wo - 1);
        const size_t pix = (((size_t)b << s.lW) + 2 * yq + py) * s.W + 2 * xq + px;
        const size_t q = (pix << s.lCin) + n;
        dprev[q] = to_bf16(from_bf16(prev[q]) > 0.0f ? v : 0.0f);
    }
    static constexpr bool STORE8 = true;
    __device__ __bf16 pre(int, int, float v) const { return to_bf16(v); }
    __device__ void store8(int m, int n, bf16x8 v) const {
        const int b = m >> (2 * s.lWo), r = m & ((1 << (2 * s.lWo)) - 1);
        const int yq = r >> s.lWo, xq = r & (s.Wo - 1);
        const size_t pix = (((size_t)b << s.lW) + 2 * yq + py) * s.W + 2 * xq + px;
        const size_t q = (pix << s.lCin) + n;
        *reinterpret_cast<bf16x8*>(dprev + q) = relu_mask8(v, ld8(prev + q));
    }
};

// The four parity classes of OpConvDgradS2 in one launch (gridDim.z = 4,
// class c = 2 py + px, K = taps(c) Cout), so that the classes of one output
// tile, which read the same dZ rows, run back to back on one XCD.
struct OpConvDgradS2All : OpConvDgradS2 {
    static constexpr bool CLASSES = true;
    __device__ void set_class(int c) {
        py = c >> 1;
        px = c & 1;
    }
    __device__ int class_k() const { return ((py ? 2 : 1) * (px ? 2 : 1)) << s.lCout; }
};

// weight gradient (split over K = B*Ho*Wo): dW[co][tap*Cin+ci] partial per split.
// A(m = co, k = pos) = dZ[pos][co]: K-major; B(k = pos, n = (tap, ci)) =
// in[b, s y + ky - 1, s x + kx - 1, ci]: K-major when Cin >= 8, else gathered.
struct OpConvWgrad {
    static constexpr bool A_KMAJOR = true, B_KMAJOR = true;
    ConvShape s;
    const __bf16* dz;   // [B*Ho*Wo][Cout]
    const __bf16* in;   // layer input [B][H][W][Cin]
    float* part;        // [splits][Cout][9*Cin]
    // gathers of B: Cin >= 8 (the first layer has its own kernel)
    static constexpr bool CTX_A = false, CTX_B = true;
    static constexpr bool STORE8 = false;
    __device__ WRow b_row(int n) const {
        if (n >= 9 * s.Cin) return WRow{0, -100, 0};
        const int tap = n >> s.lCin, ky = div3(tap), kx = tap - 3 * ky;
        return WRow{((ky - 1) * s.W + (kx - 1)) * s.Cin + (n & (s.Cin - 1)), ky - 1, kx - 1};
    }
    __device__ WPos b_pos(int k) const {
        const int b = k >> (2 * s.lWo), r = k & ((1 << (2 * s.lWo)) - 1);
        const int iy = (r >> s.lWo) * s.stride, ix = (r & (s.Wo - 1)) * s.stride;
        return WPos{((b * s.H + iy) * s.W + ix) * s.Cin, iy, ix};
    }
    __device__ bf16x8 b_load(const WRow& w, const WPos& p) const {
        const int iy = p.iy + w.dy, ix = p.ix + w.dx;
        return ((unsigned)iy < (unsigned)s.H && (unsigned)ix < (unsigned)s.W) ? ld8(in + p.base + w.off) : zero8();
    }
    __device__ bf16x8 loadAT(int k, int m) const {
        return m < s.Cout ? ld8(dz + ((size_t)k << s.lCout) + m) : zero8();
    }
    __device__ bf16x8 loadBT(int k, int n) const {
        const int b = k >> (2 * s.lWo), r = k & ((1 << (2 * s.lWo)) - 1);
        const int y = r >> s.lWo, x = r & (s.Wo - 1);
        bf16x8 v = zero8();
        if (s.Cin >= 8) {
            if (n >= 9 * s.Cin) return v;
            const int tap = n >> s.lCin, ci = n & (s.Cin - 1), ky = div3(tap);
            const int iy = y * s.stride + ky - 1, ix = x * s.stride + (tap - 3 * ky) - 1;
            if (iy < 0 || iy >= s.H || ix < 0 || ix >= s.W) return v;
            return ld8(in + ((((size_t)b << s.lW) + iy) << s.lW) * s.Cin + ((size_t)ix << s.lCin) + ci);
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {   // Cin = 1: n is the tap
            const int tap = n + q;
            if (tap >= 9) break;
            const int ky = div3(tap);
            const int iy = y * s.stride + ky - 1, ix = x * s.stride + (tap - 3 * ky) - 1;
            if (iy >= 0 && iy < s.H && ix >= 0 && ix < s.W) v[q] = in[(((size_t)b << s.lW) + iy) * s.W + ix];
        }
        return v;
    }
    __device__ void store(int m, int n, float v, int split) const {
        part[((size_t)split * s.Cout + m) * 9 * s.Cin + n] = v;
    }
};

// fully connected forward: y[b][n] = act(sum_k x[b][k] W[n][k] + bias[n])
struct OpFcFwd {
    static constexpr bool A_KMAJOR = false, B_KMAJOR = false;
    static constexpr bool CTX_A = false, CTX_B = false;
    static constexpr bool STORE8 = false;
    int In, Out, relu;
    const __bf16* x;
    const __bf16* w;
    const float* bias;
    __bf16* ybf;     // bf16 output (hidden layer) or null
    float* yf;       // fp32 output (final layer) or null
    __device__ bf16x8 loadA(int m, int k, int kend) const {
        return k < kend ? ld8(x + (size_t)m * In + k) : zero8();
    }
    __device__ bf16x8 loadB(int k, int n, int kend) const {
        return k < kend ? ld8(w + (size_t)n * In + k) : zero8();
    }
    __device__ void store(int m, int n, float v, int) const {
        float y = v + bias[n];
        if (relu) y = fmaxf(y, 0.0f);
        if (ybf) ybf[(size_t)m * Out + n] = to_bf16(y);
        if (yf) yf[(size_t)m * Out + n] = y;
    }
};

// fully connected data gradient: dx[b][k] = sum_n dy[b][n] W[n][k], masked by x > 0
// (mask_src null: no mask, output fp32).  A(m = b, k = out) = dy[b][out]
// along K; B(k = out, n = in) = W[out][in]: K-major.
struct OpFcDgrad {
    static constexpr bool A_KMAJOR = false, B_KMAJOR = true;
    static constexpr bool CTX_A = false, CTX_B = false;
    static constexpr bool STORE8 = false;
    int In, Out;
    const __bf16* dy;     // [B][Out]
    const __bf16* w;      // [Out][In]
    const __bf16* mask_src;
    __bf16* dxbf;
    float* dxf;
    __device__ bf16x8 loadA(int m, int k, int kend) const {
        bf16x8 v = zero8();
        if ((Out & 7) == 0) return k < kend ? ld8(dy + (size_t)m * Out + k) : v;
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (k + q < kend) v[q] = dy[(size_t)m * Out + k + q];
        return v;
    }
    __device__ bf16x8 loadBT(int k, int n) const { return n < In ? ld8(w + (size_t)k * In + n) : zero8(); }
    __device__ void store(int m, int n, float v, int) const {
        const size_t q = (size_t)m * In + n;
        if (mask_src && !(from_bf16(mask_src[q]) > 0.0f)) v = 0.0f;
        if (dxbf) dxbf[q] = to_bf16(v);
        if (dxf) dxf[q] = v;
    }
};

// fully connected weight gradient: dW[n][k] = sum_b dy[b][n] x[b][k].
// A(m = out, k = b) = dy[b][out], B(k = b, n = in) = x[b][in]: both K-major.
struct OpFcWgrad {
    static constexpr bool A_KMAJOR = true, B_KMAJOR = true;
    static constexpr bool CTX_A = false, CTX_B = false;
    static constexpr bool STORE8 = false;
    int In, Out;
    const __bf16* dy;   // [B][Out]
    const __bf16* x;    // [B][In]
    float* dw;          // [Out][In]
    __device__ bf16x8 loadAT(int k, int m) const {
        bf16x8 v = zero8();
        if ((Out & 7) == 0) return m < Out ? ld8(dy + (size_t)k * Out + m) : v;
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (m + q < Out) v[q] = dy[(size_t)k * Out + m + q];
        return v;
    }
    __device__ bf16x8 loadBT(int k, int n) const { return n < In ? ld8(x + (size_t)k * In + n) : zero8(); }
    __device__ void store(int m, int n, float v, int) const { dw[(size_t)m * In + n] = v; }
};

template <class Op>
static hipError_t gemm(const Op& op, int M, int N, int K, int splits, hipStream_t st) {
    const int kps = ((K + splits - 1) / splits + GK - 1) / GK * GK;
    const int nz = (K + kps - 1) / kps;
    hipLaunchKernelGGL(k_gemm<Op>, dim3((M + GT - 1) / GT, (N + GT - 1) / GT, nz), dim3(256), 0, st, op,
                       M, N, K, kps);
    return hipGetLastError();
}

// Large-M GEMM (no K split): the 128 x 64 tile.
template <class Op>
static hipError_t gemm_tall(const Op& op, int M, int N, int K, hipStream_t st) {
    hipLaunchKernelGGL(k_gemm_tall<Op>, dim3((M + GT2 - 1) / GT2, (N + GT - 1) / GT, 1), dim3(256), 0, st, op, M,
                       N, K, K);
    return hipGetLastError();
}

// Picks the tile for a GEMM shape: the 64 x 64-per-wave tiles where the
// output is large enough in both directions to fill them, 256 x 32 for
// 32-column outputs, else the tall (large M, no split) or the square 64 x 64
// kernel.
template <class Op>
static hipError_t gemm_pick(const Op& op, int M, int N, int K, int splits, hipStream_t st) {
    const int kps = ((K + splits - 1) / splits + GK - 1) / GK * GK;
    const int nz = (K + kps - 1) / kps;
    if (M >= 128 && N >= 128) {
        hipLaunchKernelGGL((k_gemm_wide<Op, 2, 2>), dim3((M + 127) / 128, (N + 127) / 128, nz), dim3(256), 0, st, op,
                           M, N, K, kps);
    } else if (N >= 64 && M >= 256) {
        hipLaunchKernelGGL((k_gemm_wide<Op, 4, 1>), dim3((M + 255) / 256, (N + 63) / 64, nz), dim3(256), 0, st, op, M,
                           N, K, kps);
    } else if (M >= 64 && N >= 512) {
        hipLaunchKernelGGL((k_gemm_wide<Op, 1, 4>), dim3((M + 63) / 64, (N + 255) / 256, nz), dim3(256), 0, st, op, M,
                           N, K, kps);
    } else if (N <= 32 && M >= 256) {
        hipLaunchKernelGGL((k_gemm_wide<Op, 4, 1, 2>), dim3((M + 255) / 256, 1, nz), dim3(256), 0, st, op, M, N, K,
                           kps);
    } else if (nz == 1 && M >= 4096) {
        return gemm_tall(op, M, N, K, st);
    } else {
        return gemm(op, M, N, K, splits, st);
    }
    return hipGetLastError();
}

// One launch over nc classes of an op with CLASSES, for outputs of at most
// 32 columns (the 256 x 32 tile, no K split); false for other shapes, whose
// classes the caller launches one by one.  Measured on the network's
// stride-2 data gradients at batch 1024: the first (32 channels, 64 x 64
// output) 265 -> 219 us in one launch; the 64- and 128-channel ones gain
// nothing (135 -> 133 us) or lose (79 -> 87 us) with their wider tiles.
template <class Op>
static bool gemm_classes(const Op& op, int M, int N, int nc, hipStream_t st) {
    if (!(N <= 32 && M >= 256)) return false;
    hipLaunchKernelGGL((k_gemm_wide<Op, 4, 1, 2>), dim3((M + 255) / 256, 1, nc), dim3(256), 0, st, op, M, N, 0, 0);
    return true;
}

static int gemm_splits(int M, int N, int K, int splits) {
    const int kps = ((K + splits - 1) / splits + GK - 1) / GK * GK;
    return (K + kps - 1) / kps;
}

// ---------------------------------------------------------------------------
// First convolution (one input channel, 3 x 3, CNN_C1 = 32 outputs, stride 1)
// as direct VALU kernels: K = 9 is too short for the matrix cores, and the
// GEMM path pads it to 32 and gathers single bf16 values.  One work-group
// per image; the image (zero border) is staged in LDS as float; thread
// t = 4 x + g handles pixel column x and output channels 8 g .. 8 g + 7, one
// image row at a time, so a wave's 16-byte accesses of the NHWC activation
// rows are contiguous.
// ---------------------------------------------------------------------------
constexpr int C0_OUT = 32;
constexpr int C0_SIDE = CNN_IN + 2;   // 66: image plus a zero border

__device__ __forceinline__ void c0_stage_image(const __bf16* __restrict__ img, float (*tile)[C0_SIDE]) {
    for (int q = threadIdx.x; q < C0_SIDE * C0_SIDE; q += blockDim.x) {
        const int y = q / C0_SIDE - 1, x = q % C0_SIDE - 1;
        tile[y + 1][x + 1] = (y >= 0 && y < CNN_IN && x >= 0 && x < CNN_IN) ? from_bf16(img[y * CNN_IN + x]) : 0.0f;
    }
}

// out[b, y, x, co] = relu(sum_tap W[co][tap] in[b, y + ky - 1, x + kx - 1] + bias[co]) as bf16;
// the tap sum in float, in tap order, then the bias (the GEMM epilogue's order).
__global__ __launch_bounds__(256) void k_conv0_fwd(const __bf16* __restrict__ img, const __bf16* __restrict__ w,
                                                   const float* __restrict__ bias, __bf16* __restrict__ out) {
    __shared__ float tile[C0_SIDE][C0_SIDE];
    const int b = blockIdx.x;
    const int t = threadIdx.x, g = t & 3, x = t >> 2;
    c0_stage_image(img + (size_t)b * CNN_IN * CNN_IN, tile);
    float wr[8][9], br[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
#pragma unroll
        for (int q = 0; q < 9; ++q) wr[c][q] = from_bf16(w[(8 * g + c) * 9 + q]);
        br[c] = bias[8 * g + c];
    }
    __syncthreads();
    __bf16* o = out + ((size_t)b * CNN_IN * CNN_IN) * C0_OUT + 8 * g;
    for (int y = 0; y < CNN_IN; ++y) {
        float v[9];
#pragma unroll
        for (int ky = 0; ky < 3; ++ky)
#pragma unroll
            for (int kx = 0; kx < 3; ++kx) v[3 * ky + kx] = tile[y + ky][x + kx];
        bf16x8 r;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            float a = 0.0f;
#pragma unroll
            for (int q = 0; q < 9; ++q) a = fmaf(wr[c][q], v[q], a);
            r[c] = to_bf16(fmaxf(a + br[c], 0.0f));
        }
        *reinterpret_cast<bf16x8*>(o + ((size_t)y * CNN_IN + x) * C0_OUT) = r;
    }
}

// Rows r and r + 1 of the zero-bordered image as bf16 pairs: pairs[r][c] =
// (tile[r][c], tile[r + 1][c]) in the low and high halves, tile row r being
// image row r - 1 (the staging of c0_stage_image, two rows at once).
__device__ __forceinline__ void c0_stage_pairs(const __bf16* __restrict__ img, uint32_t (*pairs)[C0_SIDE]) {
    auto px = [&](int y, int x) -> uint32_t {
        return (y >= 0 && y < CNN_IN && x >= 0 && x < CNN_IN)
                   ? (uint32_t)__builtin_bit_cast(unsigned short, img[y * CNN_IN + x])
                   : 0u;
    };
    for (int q = threadIdx.x; q < (C0_SIDE - 1) * C0_SIDE; q += blockDim.x) {
        const int r = q / C0_SIDE, c = q % C0_SIDE;
        pairs[r][c] = px(r - 1, c - 1) | (px(r, c - 1) << 16);
    }
}

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// a.x b.x + a.y b.y + c (bf16 products are exact in float)
__device__ __forceinline__ float dot2(uint32_t a, uint32_t b, float c) {
    return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, a), __builtin_bit_cast(bf16x2, b), c, false);
}

// Per image b: part[b][co][q] = sum over pixels of dZ[b, y, x, co] times
// in[b, y + ky - 1, x + kx - 1] (q = 3 ky + kx < 9) or times 1 (q = 9: the
// bias gradient).  Thread t = 4 x + g takes pixel column x and channels
// 8 g .. 8 g + 7 and sums its 64 rows in float, two rows at a time: each
// pair of products (row y, row y + 1) is one bf16 dot instruction.  The 16
// pixel columns of a wave are combined by a fixed butterfly, the four waves
// in LDS in float64, in fixed order.
__global__ __launch_bounds__(256) void k_conv0_wgrad(const __bf16* __restrict__ img, const __bf16* __restrict__ dz,
                                                     double* __restrict__ part) {
    __shared__ uint32_t pairs[C0_SIDE - 1][C0_SIDE];
    __shared__ double red[4][C0_OUT * 10];
    const int b = blockIdx.x;
    const int t = threadIdx.x, g = t & 3, x = t >> 2, lane = t & 63, wv = t >> 6;
    c0_stage_pairs(img + (size_t)b * CNN_IN * CNN_IN, pairs);
    __syncthreads();
    float acc[8][10];
#pragma unroll
    for (int c = 0; c < 8; ++c)
#pragma unroll
        for (int q = 0; q < 10; ++q) acc[c][q] = 0.0f;
    const __bf16* d = dz + ((size_t)b * CNN_IN * CNN_IN) * C0_OUT + 8 * g + (size_t)x * C0_OUT;
    // the 16 bytes of row y + PF are requested before row y's products (a
    // ring of PF rows in flight; one work-group per image leaves few waves
    // per SIMD to hide the latency)
    constexpr int PF = 4;
    constexpr size_t ROW = (size_t)CNN_IN * C0_OUT;
    constexpr uint32_t ONES = 0x3F803F80u;   // bf16 (1, 1)
    bf16x8 ring[PF];
#pragma unroll
    for (int q = 0; q < PF; ++q) ring[q] = *reinterpret_cast<const bf16x8*>(d + q * ROW);
    for (int y0 = 0; y0 < CNN_IN; y0 += PF) {
#pragma unroll
        for (int q = 0; q < PF; q += 2) {
            const int y = y0 + q;
            const bf16x8 d0 = ring[q], d1 = ring[q + 1];
            if (y + PF < CNN_IN) {
                ring[q] = *reinterpret_cast<const bf16x8*>(d + (y + PF) * ROW);
                ring[q + 1] = *reinterpret_cast<const bf16x8*>(d + (y + 1 + PF) * ROW);
            }
            uint32_t v[9];
#pragma unroll
            for (int ky = 0; ky < 3; ++ky)
#pragma unroll
                for (int kx = 0; kx < 3; ++kx) v[3 * ky + kx] = pairs[y + ky][x + kx];
            const uint32_t* w0 = reinterpret_cast<const uint32_t*>(&d0);
            const uint32_t* w1 = reinterpret_cast<const uint32_t*>(&d1);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                // channels 2k and 2k + 1 of rows y and y + 1 as (row y, row y + 1) pairs
                const uint32_t lo = __builtin_amdgcn_perm(w1[k], w0[k], 0x05040100u);
                const uint32_t hi = __builtin_amdgcn_perm(w1[k], w0[k], 0x07060302u);
#pragma unroll
                for (int r = 0; r < 9; ++r) {
                    acc[2 * k][r] = dot2(lo, v[r], acc[2 * k][r]);
                    acc[2 * k + 1][r] = dot2(hi, v[r], acc[2 * k + 1][r]);
                }
                acc[2 * k][9] = dot2(lo, ONES, acc[2 * k][9]);
                acc[2 * k + 1][9] = dot2(hi, ONES, acc[2 * k + 1][9]);
            }
        }
    }
    // lanes 4 j + g (j = 0..15) of a wave hold the same channels: butterfly over j
#pragma unroll
    for (int c = 0; c < 8; ++c)
#pragma unroll
        for (int q = 0; q < 10; ++q) {
            float a = acc[c][q];
#pragma unroll
            for (int off = 4; off < 64; off <<= 1) a += __shfl_xor(a, off, 64);
            acc[c][q] = a;
        }
    if (lane < 4) {
#pragma unroll
        for (int c = 0; c < 8; ++c)
#pragma unroll
            for (int q = 0; q < 10; ++q) red[wv][(8 * g + c) * 10 + q] = (double)acc[c][q];
    }
    __syncthreads();
    for (int e = t; e < C0_OUT * 10; e += blockDim.x)
        part[(size_t)b * C0_OUT * 10 + e] = ((red[0][e] + red[1][e]) + red[2][e]) + red[3][e];
}

// dW and db of the first convolution: sum over the B images of part, one wave
// per entry (lane l sums images l, l + 64, ...; a fixed butterfly combines).
__global__ __launch_bounds__(256) void k_conv0_wgrad_final(int B, const double* __restrict__ part,
                                                           float* __restrict__ dw, float* __restrict__ db) {
    const int e = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (e >= C0_OUT * 10) return;
    double s = 0.0;
    for (int b = lane; b < B; b += 64) s += part[(size_t)b * C0_OUT * 10 + e];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) {
        const int co = e / 10, q = e % 10;
        if (q < 9) dw[co * 9 + q] = (float)s;
        else db[co] = (float)s;
    }
}

// ---------------------------------------------------------------------------
// Elementwise / reduction kernels
// ---------------------------------------------------------------------------
// sum of split-K partials in fixed order: out[i] = sum_z part[z][i]
__global__ void k_sum_splits(int nz, long long n, const float* __restrict__ part, float* __restrict__ out) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int z = 0; z < nz; ++z) s += part[(size_t)z * n + i];
    out[i] = (float)s;
}

// The same for many splits, read coalesced: a work-group of 64 G threads
// takes 64 consecutive outputs; wave g sums splits [g zc, (g + 1) zc) in
// order (64 consecutive floats per split row), then the G wave sums are
// added in g order.  Each output's order is fixed by (nz, zc).
__global__ __launch_bounds__(1024) void k_sum_splits_cols(int nz, int zc, long long n,
                                                          const float* __restrict__ part, float* __restrict__ out) {
    __shared__ double red[16][64];
    const int lane = threadIdx.x & 63, g = threadIdx.x >> 6, G = blockDim.x >> 6;
    const long long i = (long long)blockIdx.x * 64 + lane;
    double s = 0.0;
    if (i < n) {
        const int z1 = min(nz, (g + 1) * zc);
#pragma unroll 8
        for (int z = g * zc; z < z1; ++z) s += part[(size_t)z * n + i];
    }
    red[g][lane] = s;
    __syncthreads();
    if (g == 0 && i < n) {
        double t = red[0][lane];
        for (int q = 1; q < G; ++q) t += red[q][lane];
        out[i] = (float)t;
    }
}

// column sums of a bf16 matrix [rows][cols] (bias gradients), fixed order:
// stage 1 partial[chunk][col], stage 2 sums the chunks.
__global__ void k_colsum_partial(int rows, int cols, int rows_per_chunk, const __bf16* __restrict__ x,
                                 double* __restrict__ part) {
    const int col = blockIdx.x * 64 + (threadIdx.x & 63);
    const int sub = threadIdx.x >> 6;   // 0..3
    const int r0 = blockIdx.y * rows_per_chunk, r1 = min(rows, r0 + rows_per_chunk);
    __shared__ double red[4][64];
    double s = 0.0;
    if (col < cols)
        for (int r = r0 + sub; r < r1; r += 4) s += (double)from_bf16(x[(size_t)r * cols + col]);
    red[sub][threadIdx.x & 63] = s;
    __syncthreads();
    if (sub == 0 && col < cols)
        part[(size_t)blockIdx.y * cols + col] =
            (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
}

// The same for cols a multiple of 8 (<= 2048), read row-major 16 bytes per
// thread (coalesced): thread t sums column group t % (cols/8) over rows
// t / (cols/8), + 256/(cols/8), ...; the per-thread sums are combined in LDS
// in fixed order.
__global__ __launch_bounds__(256) void k_colsum8_partial(int rows, int cols, int rows_per_chunk,
                                                         const __bf16* __restrict__ x, double* __restrict__ part) {
    __shared__ double red[2048];
    const int g = cols >> 3, per = 256 / g;
    const int t = threadIdx.x, cg = t % g, ro = t / g;
    const int r0 = blockIdx.x * rows_per_chunk, r1 = min(rows, r0 + rows_per_chunk);
    double acc[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] = 0.0;
    if (ro < per)
        for (int r = r0 + ro; r < r1; r += per) {
            const bf16x8 v = *reinterpret_cast<const bf16x8*>(x + (size_t)r * cols + cg * 8);
#pragma unroll
            for (int i = 0; i < 8; ++i) acc[i] += (double)from_bf16(v[i]);
        }
    if (ro < per)
#pragma unroll
        for (int i = 0; i < 8; ++i) red[ro * cols + cg * 8 + i] = acc[i];
    __syncthreads();
    for (int c = t; c < cols; c += 256) {
        double sum = 0.0;
        for (int q = 0; q < per; ++q) sum += red[q * cols + c];
        part[(size_t)blockIdx.x * cols + c] = sum;
    }
}

// out[c] = sum over chunks of part[chunk][c]: one wave per column, lane l
// sums chunks l, l + 64, ..., then a fixed butterfly combines the lanes.
__global__ __launch_bounds__(256) void k_colsum_final(int chunks, int cols, const double* __restrict__ part,
                                                      float* __restrict__ out) {
    const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (c >= cols) return;
    double s = 0.0;
    for (int z = lane; z < chunks; z += 64) s += part[(size_t)z * cols + c];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) out[c] = (float)s;
}

// global average pool over HxW of a [B][H][W][C] bf16 tensor -> bf16 [B][C]
__global__ void k_pool_fwd(int B, int HW, int C, const __bf16* __restrict__ x, __bf16* __restrict__ y) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= B * C) return;
    const int b = q / C, c = q - b * C;
    float s = 0.0f;
    for (int p = 0; p < HW; ++p) s += from_bf16(x[((size_t)b * HW + p) * C + c]);
    y[q] = to_bf16(s / (float)HW);
}

// pooling backward with the ReLU mask of the pooled activation: dz = dy/HW * (x > 0)
__global__ void k_pool_bwd(int B, int HW, int C, const float* __restrict__ dy, const __bf16* __restrict__ x,
                           __bf16* __restrict__ dz) {
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (long long)B * HW * C) return;
    const int c = (int)(q % C);
    const int b = (int)(q / ((long long)HW * C));
    const float g = dy[(size_t)b * C + c] / (float)HW;
    dz[q] = to_bf16(from_bf16(x[q]) > 0.0f ? g : 0.0f);
}

// Gaussian negative log-likelihood per sample, mean over the batch:
//   L = 1/B sum_b sum_j [ (z - mu)^2 exp(-s) / 2 + s / 2 ],  out = [mu(NT), s(NT)]
// d out written as bf16 (input of the last layer's backward GEMMs).
__global__ void k_nll(int B, const float* __restrict__ out, const float* __restrict__ target,
                      __bf16* __restrict__ dout, double* __restrict__ loss_part) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    double l = 0.0;
    if (b < B) {
        for (int j = 0; j < CNN_NT; ++j) {
            const float mu = out[(size_t)b * CNN_OUT + j], s = out[(size_t)b * CNN_OUT + CNN_NT + j];
            const float z = target[(size_t)b * CNN_NT + j];
            const float e = expf(-s), r = z - mu;
            l += 0.5 * (double)(r * r * e) + 0.5 * (double)s;
            dout[(size_t)b * CNN_OUT + j] = to_bf16(-r * e / (float)B);
            dout[(size_t)b * CNN_OUT + CNN_NT + j] = to_bf16(0.5f * (1.0f - r * r * e) / (float)B);
        }
    }
    __shared__ double red[256];
    red[threadIdx.x] = l;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0];
}

__global__ void k_loss_final(int nb, int B, const double* __restrict__ part, float* __restrict__ loss) {
    double s = 0.0;
    for (int i = 0; i < nb; ++i) s += part[i];
    *loss = (float)(s / B);
}

// Adam on the fp32 master parameters; refreshes the bf16 copies of weights.
// The learning rate and the (1-based) step come from device memory
// (hyper = {lr, step}), so that a captured training step serves every step.
__global__ void k_cnn_adam(long long n, float* __restrict__ p, const float* __restrict__ g,
                           float* __restrict__ m, float* __restrict__ v, __bf16* __restrict__ pbf,
                           const float* __restrict__ hyper, float b1, float b2, float eps) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float lr = hyper[0];
    const int step = (int)hyper[1];
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / (1.0f - powf(b1, (float)step));
    const float vh = vi / (1.0f - powf(b2, (float)step));
    const float pi = p[i] - lr * mh / (sqrtf(vh) + eps);
    p[i] = pi;
    pbf[i] = to_bf16(pi);
}

__global__ void k_to_bf16(long long n, const float* __restrict__ x, __bf16* __restrict__ y) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = to_bf16(x[i]);
}

// Random numbers: Philox4x32-10 of lens_philox.h (initial weights, noise, proposals).
__device__ __forceinline__ uint4 philox_c(uint4 c, uint2 k) { return philox4x32_10(c, k); }
__device__ __forceinline__ double unif(uint32_t w) { return philox_uniform01(w); }

// standard normal from counter (a, b, c): Box-Muller on words 0, 1
__device__ __forceinline__ double normal_at(uint64_t seed, uint32_t a, uint32_t b, uint32_t c) {
    const uint4 w = philox_c(make_uint4(a, b, c, 0x5eedu), make_uint2((uint32_t)seed, (uint32_t)(seed >> 32)));
    return sqrt(-2.0 * log(unif(w.x))) * cos(6.283185307179586476925 * unif(w.y));
}

// He-normal initialisation of the weights of one tensor (fan_in), zero biases
__global__ void k_init_normal(long long n, float scale, uint64_t seed, uint32_t tensor, float* __restrict__ p) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    p[i] = (float)(scale * normal_at(seed, (uint32_t)i, tensor, 1u));
}

// Noise, asinh(x / (3 sigma)) transform and bf16 rounding of simulated images
__global__ void k_prepare(long long n, const float* __restrict__ img, float sigma, int add_noise, uint64_t seed,
                          uint64_t counter0, __bf16* __restrict__ out) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double x = img[i];
    if (add_noise) {
        const uint64_t c = counter0 + (uint64_t)i;
        x += sigma * normal_at(seed, (uint32_t)c, (uint32_t)(c >> 32), 2u);
    }
    out[i] = to_bf16((float)asinh(x / (3.0 * sigma)));
}

// ---------------------------------------------------------------------------
// Proposals: CNN Gaussian for the mapped parameters, prior draws for the rest
// ---------------------------------------------------------------------------
__device__ double ndtri_d(double p) { return 1.4142135623730951 * erfinv(2.0 * p - 1.0); }
__device__ double ndtr_d(double z) { return 0.5 * erfc(-z * 0.7071067811865476); }
// the same inverse for small p (no loss in 2p - 1): -sqrt(2) erfcinv(2p)
__device__ double ndtri_lo(double p) { return -1.4142135623730951 * erfcinv(2.0 * p); }

// One thread per proposal (system s0 + s, draw i); counters use the global
// system index so that chunked calls draw the same numbers.
// A draw from prior row (kind, a, b, lo, hi) by inverse CDF of u in (0, 1).
__device__ double prior_draw(int kind, double a, double b, double lo, double hi, double u) {
    if (kind == LENS_PRIOR_UNIFORM) return a + (b - a) * u;
    if (kind == LENS_PRIOR_NORMAL) return a + b * ndtri_d(u);
    if (kind == LENS_PRIOR_LOGNORMAL) return exp(a + b * ndtri_d(u));
    const double pl = ndtr_d((lo - a) / b), ph = ndtr_d((hi - a) / b);
    return a + b * ndtri_d(pl + u * (ph - pl));
}

__global__ void k_propose(int S, int s0, int n, int d, const float* __restrict__ net_out,
                          const CnnTargetMap* __restrict__ tm, uint64_t seed, float* __restrict__ theta,
                          int* __restrict__ flags) {
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (long long)S * n) return;
    const int s = (int)(q / n), i = (int)(q - (long long)s * n);
    const uint32_t sg = (uint32_t)(s0 + s);
    float* th = theta + (size_t)q * d;
    int clipped = 0;
    for (int j = 0; j < d; ++j) {
        const int kind = tm->prior_kind[j];
        const double a = tm->prior[j][0], b = tm->prior[j][1], lo = tm->prior[j][2], hi = tm->prior[j][3];
        const int c = tm->cnn_slot[j];
        double v;
        if (c >= 0) {
            // the network's Gaussian N(m, sd^2) truncated to the prior's support,
            // drawn by inverse CDF on tail probabilities when the support lies
            // in a tail (so that they stay accurate); the system is flagged
            // when the truncation removes more than 1 % of the mass
            const double mu = net_out[(size_t)s * CNN_OUT + c];
            const double ls = fmin(fmax((double)net_out[(size_t)s * CNN_OUT + CNN_NT + c], -30.0), 10.0);
            const double m = tm->mean[c] + tm->stdv[c] * mu, sd = tm->stdv[c] * exp(0.5 * ls);
            double vlo = -INFINITY, vhi = INFINITY;
            if (kind == LENS_PRIOR_UNIFORM) { vlo = a; vhi = b; }
            else if (kind == LENS_PRIOR_TRUNCNORMAL) { vlo = lo; vhi = hi; }
            else if (kind == LENS_PRIOR_LOGNORMAL) { vlo = 0.0; }
            const double al = (vlo - m) / sd, be = (vhi - m) / sd;
            const uint4 w = philox_c(make_uint4(sg, (uint32_t)i, 16u + (uint32_t)j, 0x7e1u),
                                     make_uint2((uint32_t)seed, (uint32_t)(seed >> 32)));
            const double u = unif(w.x);
            double z, mass;
            if (be < 0.0) {            // support in the lower tail: small probabilities
                const double pa = ndtr_d(al), pb = ndtr_d(be);
                mass = pb - pa;
                z = ndtri_lo(pa + u * mass);
            } else if (al > 0.0) {     // upper tail, by symmetry
                const double pa = ndtr_d(-be), pb = ndtr_d(-al);
                mass = pb - pa;
                z = -ndtri_lo(pa + u * mass);
            } else {                   // the support holds the mean
                const double pa = ndtr_d(al), pb = ndtr_d(be);
                mass = pb - pa;
                z = ndtri_d(pa + u * mass);
            }
            if (!(mass >= 0.99)) clipped = 1;
            if (mass >= 0.5) {
                v = m + sd * z;
                // rounding guard: keep the draw strictly inside the support
                const double eps = 1e-9 * (vhi - vlo < INFINITY ? (vhi - vlo) : 1.0);
                v = fmin(fmax(v, vlo + eps), vhi - eps);
            } else {
                // the network's Gaussian lies mostly outside the support (its
                // truncation would hug the bound): a prior draw instead
                v = prior_draw(kind, a, b, lo, hi, u);
            }
        } else {
            const uint4 w = philox_c(make_uint4(sg, (uint32_t)i, 64u + (uint32_t)j, 0x9a1u),
                                     make_uint2((uint32_t)seed, (uint32_t)(seed >> 32)));
            v = prior_draw(kind, a, b, lo, hi, unif(w.x));
        }
        th[j] = (float)v;
    }
    if (flags && clipped) atomicOr(flags + s, 1);
}

__global__ void k_zero_int(int n, int* __restrict__ x) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = 0;
}

// ---------------------------------------------------------------------------
// Network: forward / backward / step
// ---------------------------------------------------------------------------
static inline dim3 g1(long long n, int bs = 256) { return dim3((unsigned)((n + bs - 1) / bs)); }

hipError_t cnn_forward(CnnNet& net, int B, const __bf16* img, hipStream_t st) {
    if (net.conv[0].cin != 1 || net.conv[0].cout != C0_OUT || net.conv[0].stride != 1) return hipErrorInvalidValue;
    const __bf16* x = img;
    int H = CNN_IN;
    for (int l = 0; l < CNN_CONV; ++l) {
        const CnnLayer& L = net.conv[l];
        if (l == 0) {
            hipLaunchKernelGGL(k_conv0_fwd, dim3(B), dim3(256), 0, st, x, net.wbf + L.w_off, net.params + L.b_off,
                               net.act[0]);
            x = net.act[0];
            continue;
        }
        const ConvShape s = conv_shape(B, H, L.cin, H / L.stride, L.cout, L.stride);
        OpConvFwd op{s, x, net.wbf + L.w_off, net.params + L.b_off, net.act[l]};
        if (gemm_pick(op, B * s.Ho * s.Wo, L.cout, 9 * L.cin, 1, st) != hipSuccess) return hipErrorLaunchFailure;
        x = net.act[l];
        H = s.Ho;
    }
    hipLaunchKernelGGL(k_pool_fwd, g1((long long)B * CNN_C6), dim3(256), 0, st, B, H * H, CNN_C6, x, net.pooled);
    OpFcFwd f1{CNN_C6, CNN_H1, 1, net.pooled, net.wbf + net.fc1.w_off, net.params + net.fc1.b_off, net.hidden, nullptr};
    if (gemm(f1, B, CNN_H1, CNN_C6, 1, st) != hipSuccess) return hipErrorLaunchFailure;
    OpFcFwd f2{CNN_H1, CNN_OUT, 0, net.hidden, net.wbf + net.fc2.w_off, net.params + net.fc2.b_off, nullptr, net.out};
    if (gemm(f2, B, CNN_OUT, CNN_H1, 1, st) != hipSuccess) return hipErrorLaunchFailure;
    return hipGetLastError();
}

// bias gradient = column sums of dz [rows][cols]
static hipError_t bias_grad(CnnNet& net, int rows, int cols, const __bf16* dz, float* db, hipStream_t st) {
    // chunks of rows_per_chunk rows: about 1 KB of a column group per thread
    // for tall matrices, and at least ~256 chunks (work-groups) for short ones
    const int rpc = colsum_rows_per_chunk(rows);
    const int chunks = (rows + rpc - 1) / rpc;
    if ((long long)chunks * cols > colpart_capacity(net.max_batch)) return hipErrorInvalidValue;
    if ((cols & 7) == 0 && cols <= 2048)
        hipLaunchKernelGGL(k_colsum8_partial, dim3(chunks), dim3(256), 0, st, rows, cols, rpc, dz, net.colpart);
    else
        hipLaunchKernelGGL(k_colsum_partial, dim3((cols + 63) / 64, chunks), dim3(256), 0, st, rows, cols, rpc, dz,
                           net.colpart);
    hipLaunchKernelGGL(k_colsum_final, dim3((cols + 3) / 4), dim3(256), 0, st, chunks, cols, net.colpart, db);
    return hipGetLastError();
}

hipError_t cnn_backward(CnnNet& net, int B, const __bf16* img, const float* target, float* loss, hipStream_t st) {
    const int nb = (B + 255) / 256;
    hipLaunchKernelGGL(k_nll, dim3(nb), dim3(256), 0, st, B, net.out, target, net.dout, net.losspart);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(1), 0, st, nb, B, net.losspart, loss);
    // fc2: dW, db, dhidden (masked by hidden > 0)
    OpFcWgrad w2{CNN_H1, CNN_OUT, net.dout, net.hidden, net.grads + net.fc2.w_off};
    if (gemm(w2, CNN_OUT, CNN_H1, B, 1, st) != hipSuccess) return hipErrorLaunchFailure;
    if (bias_grad(net, B, CNN_OUT, net.dout, net.grads + net.fc2.b_off, st) != hipSuccess) return hipErrorLaunchFailure;
    OpFcDgrad d2{CNN_H1, CNN_OUT, net.dout, net.wbf + net.fc2.w_off, net.hidden, net.dhidden, nullptr};
    if (gemm(d2, B, CNN_H1, CNN_OUT, 1, st) != hipSuccess) return hipErrorLaunchFailure;
    // fc1: dW, db, dpooled (fp32, pooled mask applied by the pooling backward)
    OpFcWgrad w1{CNN_C6, CNN_H1, net.dhidden, net.pooled, net.grads + net.fc1.w_off};
    if (gemm(w1, CNN_H1, CNN_C6, B, 1, st) != hipSuccess) return hipErrorLaunchFailure;
    if (bias_grad(net, B, CNN_H1, net.dhidden, net.grads + net.fc1.b_off, st) != hipSuccess) return hipErrorLaunchFailure;
    OpFcDgrad d1{CNN_C6, CNN_H1, net.dhidden, net.wbf + net.fc1.w_off, nullptr, nullptr, net.dpooled};
    if (gemm(d1, B, CNN_C6, CNN_H1, 1, st) != hipSuccess) return hipErrorLaunchFailure;
    // pooling backward into dz of the last conv layer
    const int H6 = CNN_IN / 8;
    hipLaunchKernelGGL(k_pool_bwd, g1((long long)B * H6 * H6 * CNN_C6), dim3(256), 0, st, B, H6 * H6, CNN_C6,
                       net.dpooled, net.act[CNN_CONV - 1], net.dact[CNN_CONV - 1]);
    int Hout = H6;
    for (int l = CNN_CONV - 1; l >= 0; --l) {
        const CnnLayer& L = net.conv[l];
        const int H = Hout * L.stride;
        const ConvShape s = conv_shape(B, H, L.cin, Hout, L.cout, L.stride);
        const __bf16* in = l == 0 ? img : net.act[l - 1];
        const int K = B * Hout * Hout;
        if (l == 0) {   // first layer: direct kernels (and no data gradient)
            hipLaunchKernelGGL(k_conv0_wgrad, dim3(B), dim3(256), 0, st, img, net.dact[0], net.c0part);
            hipLaunchKernelGGL(k_conv0_wgrad_final, dim3(C0_OUT * 10 / 4), dim3(256), 0, st, B, net.c0part,
                               net.grads + L.w_off, net.grads + L.b_off);
            break;
        }
        const int splits = gemm_splits(L.cout, 9 * L.cin, K, wgrad_splits(K));
        OpConvWgrad wg{s, net.dact[l], in, net.wpart};
        if (gemm_pick(wg, L.cout, 9 * L.cin, K, wgrad_splits(K), st) != hipSuccess) return hipErrorLaunchFailure;
        const long long nw = (long long)L.cout * 9 * L.cin;
        if (splits >= 64) {
            const int G = splits >= 512 ? 16 : (splits + 31) / 32, zc = (splits + G - 1) / G;
            hipLaunchKernelGGL(k_sum_splits_cols, dim3((unsigned)((nw + 63) / 64)), dim3(64 * G), 0, st, splits, zc,
                               nw, net.wpart, net.grads + L.w_off);
        } else
            hipLaunchKernelGGL(k_sum_splits, g1(nw), dim3(256), 0, st, splits, nw, net.wpart, net.grads + L.w_off);
        if (bias_grad(net, K, L.cout, net.dact[l], net.grads + L.b_off, st) != hipSuccess) return hipErrorLaunchFailure;
        if (l > 0 && L.stride == 1) {
            OpConvDgrad dg{s, net.dact[l], net.wbf + L.w_off, net.act[l - 1], net.dact[l - 1]};
            if (gemm_pick(dg, B * H * H, L.cin, 9 * L.cout, 1, st) != hipSuccess) return hipErrorLaunchFailure;
        } else if (l > 0) {
            // stride 2: the four input-parity classes, each over its 1, 2, 2 or 4 taps,
            // in one launch where the shape takes a wide tile
            OpConvDgradS2All all{};
            all.s = s;
            all.dz = net.dact[l];
            all.w = net.wbf + L.w_off;
            all.prev = net.act[l - 1];
            all.dprev = net.dact[l - 1];
            if (gemm_classes(all, B * Hout * Hout, L.cin, 4, st)) {
                if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
            } else {
                for (int py = 0; py < 2; ++py)
                    for (int px = 0; px < 2; ++px) {
                        OpConvDgradS2 dg{s, py, px, net.dact[l], net.wbf + L.w_off, net.act[l - 1], net.dact[l - 1]};
                        const int ntap = (py ? 2 : 1) * (px ? 2 : 1);
                        if (gemm_pick(dg, B * Hout * Hout, L.cin, ntap * L.cout, 1, st) != hipSuccess)
                            return hipErrorLaunchFailure;
                    }
            }
        }
        Hout = H;
    }
    return hipGetLastError();
}

__global__ void k_set_hyper(float* __restrict__ hyper, float lr, int step) {
    hyper[0] = lr;
    hyper[1] = (float)step;
}

hipError_t cnn_set_hyper(CnnNet& net, float lr, int step, hipStream_t st) {
    hipLaunchKernelGGL(k_set_hyper, dim3(1), dim3(1), 0, st, net.hyper, lr, step);
    return hipGetLastError();
}

hipError_t cnn_adam(CnnNet& net, hipStream_t st) {
    hipLaunchKernelGGL(k_cnn_adam, g1(net.nparams), dim3(256), 0, st, (long long)net.nparams, net.params, net.grads,
                       net.adam_m, net.adam_v, net.wbf, (const float*)net.hyper, 0.9f, 0.999f, 1e-8f);
    return hipGetLastError();
}

hipError_t cnn_init(CnnNet& net, uint64_t seed, hipStream_t st) {
    auto he = [&](long long off, long long n, int fan_in, uint32_t tensor) {
        hipLaunchKernelGGL(k_init_normal, g1(n), dim3(256), 0, st, n, (float)sqrt(2.0 / fan_in), seed, tensor,
                           net.params + off);
    };
    uint32_t tensor = 0;
    for (int l = 0; l < CNN_CONV; ++l) he(net.conv[l].w_off, (long long)net.conv[l].cout * 9 * net.conv[l].cin,
                                          9 * net.conv[l].cin, tensor++);
    he(net.fc1.w_off, (long long)CNN_H1 * CNN_C6, CNN_C6, tensor++);
    // small output layer: predictions start near the standardised prior mean
    hipLaunchKernelGGL(k_init_normal, g1((long long)CNN_OUT * CNN_H1), dim3(256), 0, st, (long long)CNN_OUT * CNN_H1,
                       (float)(0.1 * sqrt(1.0 / CNN_H1)), seed, tensor++, net.params + net.fc2.w_off);
    hipLaunchKernelGGL(k_to_bf16, g1(net.nparams), dim3(256), 0, st, (long long)net.nparams, net.params, net.wbf);
    return hipGetLastError();
}

hipError_t cnn_params_to_bf16(CnnNet& net, hipStream_t st) {
    hipLaunchKernelGGL(k_to_bf16, g1(net.nparams), dim3(256), 0, st, (long long)net.nparams, net.params, net.wbf);
    return hipGetLastError();
}

hipError_t cnn_prepare(long long n, const float* img, float sigma, int add_noise, uint64_t seed, uint64_t counter0,
                       __bf16* out, hipStream_t st) {
    hipLaunchKernelGGL(k_prepare, g1(n), dim3(256), 0, st, n, img, sigma, add_noise, seed, counter0, out);
    return hipGetLastError();
}

hipError_t cnn_propose(int S, int s0, int n, int d, const float* net_out, const CnnTargetMap* tm, uint64_t seed,
                       float* theta, int* flags, hipStream_t st) {
    if (flags) hipLaunchKernelGGL(k_zero_int, g1(S), dim3(256), 0, st, S, flags);
    hipLaunchKernelGGL(k_propose, g1((long long)S * n, 64), dim3(64), 0, st, S, s0, n, d, net_out, tm, seed, theta,
                       flags);
    return hipGetLastError();
}

}  // namespace lens
