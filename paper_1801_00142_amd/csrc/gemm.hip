// Batched strided GEMM on CDNA4 matrix cores: FP64 (v_mfma_f64_16x16x4f64)
// or FP32 (v_mfma_f32_16x16x4f32, FP32 accumulation).
//
// Workgroup = 4 waves (256 threads) in a 2 x 2 arrangement; each wave owns a
// (BM/2) x (BN/2) block of C made of 16 x 16 MFMA tiles.  K is consumed in
// steps of 16: the A and B tiles are staged through LDS with k as the slow
// index so that every MFMA operand read is 16 consecutive elements per lane
// group.  The next K tile is fetched into registers while the current one
// is multiplied.  Split-K partials are kept in double and reduced in a fixed
// order.
#include "internal.h"

namespace xtrg {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int BK = 16;

// One 16x16x4 MFMA step per element type.  Operand lane l holds A(i = l%16,
// k = l/16) and B(k = l/16, j = l%16).
template <typename T> struct Mfma;
template <> struct Mfma<double> {
  using acc = d4;
  static __device__ inline acc step(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // register r of lane l holds row l/16 + 4r, column l%16
  static __device__ inline int row(int lk, int r) { return lk + 4 * r; }
};
template <> struct Mfma<float> {
  using acc = f4;
  static __device__ inline acc step(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // register r of lane l holds row 4(l/16) + r, column l%16
  static __device__ inline int row(int lk, int r) { return 4 * lk + r; }
};

// One output tile (BM x BN at m0, n0) of batch / split-K slice z, for the
// plain and the grouped launches alike (the same arithmetic in the same
// order, so a problem gets the same bits either way).
template <int BM, int BN, bool TA, bool TB, typename TI, typename TO>
__device__ __forceinline__ void gemm_tile(const Gemm& g, int m0, int n0, int z, int splitk, int kchunk,
                                          double* work) {
  using MF = Mfma<TI>;
  constexpr int WM = BM / 2, WN = BN / 2;     // wave tile
  constexpr int TM = WM / 16, TN = WN / 16;   // MFMA tiles per wave
  constexpr int LA = BM * BK / 256;           // elements of A per thread per K tile
  constexpr int LB = BN * BK / 256;
  constexpr int PAD = 4;
  __shared__ TI As[BK][BM + PAD];
  __shared__ TI Bs[BK][BN + PAD];

  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  const int ks = z % splitk;
  z /= splitk;
  const int b2 = z % g.nb[2];
  const int b1 = (z / g.nb[2]) % g.nb[1];
  const int b0 = z / (g.nb[2] * g.nb[1]);
  const TI* __restrict__ A = static_cast<const TI*>(g.A) + b0 * g.sA[0] + b1 * g.sA[1] + b2 * g.sA[2];
  const TI* __restrict__ B = static_cast<const TI*>(g.B) + b0 * g.sB[0] + b1 * g.sB[1] + b2 * g.sB[2];

  const int kbeg = ks * kchunk;
  const int kend = min(g.K, kbeg + kchunk);
  const int M = g.M, N = g.N;

  TI ra[LA], rb[LB];

  auto load = [&](int k0) {
#pragma unroll
    for (int c = 0; c < LA / 4; ++c) {
      if (!TA) {            // A[m*lda + k]: thread -> (row, 4 consecutive k)
        const int m = m0 + (t >> 2) + 64 * c;
        const int k = k0 + (t & 3) * 4;
#pragma unroll
        for (int j = 0; j < 4; ++j)
          ra[4 * c + j] = (m < M && k + j < kend) ? A[(long)m * g.lda + k + j] : TI(0);
      } else {              // A[k*lda + m]: thread -> (k row, 4 consecutive m)
        const int k = k0 + (t >> 4);
        const int m = m0 + (t & 15) * 4 + 64 * c;
#pragma unroll
        for (int j = 0; j < 4; ++j)
          ra[4 * c + j] = (k < kend && m + j < M) ? A[(long)k * g.lda + m + j] : TI(0);
      }
    }
#pragma unroll
    for (int c = 0; c < LB / 4; ++c) {
      if (!TB) {            // B[k*ldb + n]
        const int k = k0 + (t >> 4);
        const int n = n0 + (t & 15) * 4 + 64 * c;
#pragma unroll
        for (int j = 0; j < 4; ++j)
          rb[4 * c + j] = (k < kend && n + j < N) ? B[(long)k * g.ldb + n + j] : TI(0);
      } else {              // B[n*ldb + k]
        const int n = n0 + (t >> 2) + 64 * c;
        const int k = k0 + (t & 3) * 4;
#pragma unroll
        for (int j = 0; j < 4; ++j)
          rb[4 * c + j] = (n < N && k + j < kend) ? B[(long)n * g.ldb + k + j] : TI(0);
      }
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int c = 0; c < LA / 4; ++c) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (!TA) As[(t & 3) * 4 + j][(t >> 2) + 64 * c] = ra[4 * c + j];
        else     As[t >> 4][(t & 15) * 4 + 64 * c + j] = ra[4 * c + j];
      }
    }
#pragma unroll
    for (int c = 0; c < LB / 4; ++c) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (!TB) Bs[t >> 4][(t & 15) * 4 + 64 * c + j] = rb[4 * c + j];
        else     Bs[(t & 3) * 4 + j][(t >> 2) + 64 * c] = rb[4 * c + j];
      }
    }
  };

  typename MF::acc acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = typename MF::acc{TI(0), TI(0), TI(0), TI(0)};

  const int lr = lane & 15, lk = lane >> 4;
  if (kbeg < kend) {
    load(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += BK) {
      __syncthreads();
      stash();
      __syncthreads();
      if (k0 + BK < kend) load(k0 + BK);
#pragma unroll
      for (int kk = 0; kk < BK / 4; ++kk) {
        TI a[TM], b[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) a[i] = As[kk * 4 + lk][wm * WM + i * 16 + lr];
#pragma unroll
        for (int j = 0; j < TN; ++j) b[j] = Bs[kk * 4 + lk][wn * WN + j * 16 + lr];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j)
            acc[i][j] = MF::step(a[i], b[j], acc[i][j]);
      }
    }
  }

  if (splitk > 1) {
    double* __restrict__ W = work + (long)ks * M * N;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int col = n0 + wn * WN + j * 16 + lr;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = m0 + wm * WM + i * 16 + MF::row(lk, r);
          if (row < M && col < N) W[(long)row * N + col] = (double)acc[i][j][r];
        }
      }
  } else {
    TO* __restrict__ C = static_cast<TO*>(g.C) + b0 * g.sC[0] + b1 * g.sC[1] + b2 * g.sC[2];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int col = n0 + wn * WN + j * 16 + lr;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = m0 + wm * WM + i * 16 + MF::row(lk, r);
          if (row < M && col < N) C[(long)row * g.ldc + col] = (TO)acc[i][j][r];
        }
      }
  }
}

// TAG only separates kernel symbols (1 = two-site overlap C_E) for profilers.
template <int BM, int BN, bool TA, bool TB, int TAG, typename TI, typename TO>
__global__ __launch_bounds__(256) void gemm_kernel(Gemm g, int splitk, int kchunk, double* work) {
  gemm_tile<BM, BN, TA, TB, TI, TO>(g, blockIdx.y * BM, blockIdx.x * BN, blockIdx.z, splitk, kchunk, work);
}

// Grouped launch: up to kGroup independent problems (one per chain of a
// batch step, each with its own shapes, strides, pointers and split-K), the
// workgroups of problem q numbered from first[q] on.
constexpr int kGroup = 8;
struct GroupItem {
  Gemm g;
  int splitk, kchunk;
  double* work;
  int tiles_n, tiles_m;
  int first;        // first workgroup of this problem
};
struct GroupArgs {
  int n;
  GroupItem it[kGroup];
};

template <int BM, int BN>
__device__ __forceinline__ int group_find(const GroupArgs& a, int blk, int* local) {
  int q = 0;
  for (int j = 1; j < a.n; ++j)
    if (blk >= a.it[j].first) q = j;
  *local = blk - a.it[q].first;
  return q;
}

template <int BM, int BN, bool TA, bool TB, int TAG, typename TI, typename TO>
__global__ __launch_bounds__(256) void gemm_group_kernel(GroupArgs a) {
  int local;
  const int q = group_find<BM, BN>(a, blockIdx.x, &local);
  const GroupItem& it = a.it[q];
  const int tn = local % it.tiles_n, tm = (local / it.tiles_n) % it.tiles_m;
  const int z = local / (it.tiles_n * it.tiles_m);
  gemm_tile<BM, BN, TA, TB, TI, TO>(it.g, tm * BM, tn * BN, z, it.splitk, it.kchunk, it.work);
}

// Split-BF16 (bf16x3) variant for float operands: every element x is split
// at staging into hi = bf16(x) and lo = bf16(x - hi) (round to nearest
// even), and the product is accumulated in FP32 on the bf16 matrix cores
// as hi*hi + hi*lo + lo*hi with gfx950's 16 x 16 x 32 bf16 product
// (v_mfma_f32_16x16x32_bf16: twice the k of the 16 x 16 x 16 form per
// instruction).  K tiles of 32; the tiles are kept in LDS as [m][k] and
// [n][k] so that each lane's 8 consecutive k are one 16-byte read.
typedef short s8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
constexpr int BK3 = 32;

__device__ inline unsigned short bf16_rne(float x) {
  const unsigned u = __float_as_uint(x);
  return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ inline void split_bf16(float x, unsigned short* hi, unsigned short* lo) {
  *hi = bf16_rne(x);
  *lo = bf16_rne(x - __uint_as_float((unsigned)*hi << 16));
}

template <int BM, int BN, bool TA, bool TB, typename TO>
__device__ __forceinline__ void gemm_bf3_tile(const Gemm& g, int m0, int n0, int z, int splitk, int kchunk,
                                              double* work) {
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int TM = WM / 16, TN = WN / 16;
  constexpr int LA = BM * BK3 / 256;          // elements of A per thread per K tile
  constexpr int LB = BN * BK3 / 256;
  constexpr int KP = BK3 + 8;                 // padded k extent (shorts): rows of 80 bytes, 16-byte aligned
  // staging maps: a thread loads 4 consecutive elements along the stored
  // row; row-major A (no transpose) takes BK3/4 threads per m, a stored
  // K x M block (transpose) takes BM/4 threads per k (likewise for B)
  constexpr int AK = BK3 / 4, AM = BM / 4, BKT = BK3 / 4, BNT = BN / 4;
  __shared__ unsigned short Ah[BM][KP], Al[BM][KP];
  __shared__ unsigned short Bh[BN][KP], Bl[BN][KP];

  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  const int ks = z % splitk;
  z /= splitk;
  const int b2 = z % g.nb[2];
  const int b1 = (z / g.nb[2]) % g.nb[1];
  const int b0 = z / (g.nb[2] * g.nb[1]);
  const float* __restrict__ A = static_cast<const float*>(g.A) + b0 * g.sA[0] + b1 * g.sA[1] + b2 * g.sA[2];
  const float* __restrict__ B = static_cast<const float*>(g.B) + b0 * g.sB[0] + b1 * g.sB[1] + b2 * g.sB[2];

  const int kbeg = ks * kchunk;
  const int kend = min(g.K, kbeg + kchunk);
  const int M = g.M, N = g.N;

  float ra[LA], rb[LB];
  auto load = [&](int k0) {
#pragma unroll
    for (int c = 0; c < LA / 4; ++c) {
      if (!TA) {
        const int m = m0 + t / AK + (256 / AK) * c;
        const int k = k0 + (t % AK) * 4;
#pragma unroll
        for (int j = 0; j < 4; ++j) ra[4 * c + j] = (m < M && k + j < kend) ? A[(long)m * g.lda + k + j] : 0.f;
      } else {
        const int k = k0 + t / AM + (256 / AM) * c;
        const int m = m0 + (t % AM) * 4;
#pragma unroll
        for (int j = 0; j < 4; ++j) ra[4 * c + j] = (k < kend && m + j < M) ? A[(long)k * g.lda + m + j] : 0.f;
      }
    }
#pragma unroll
    for (int c = 0; c < LB / 4; ++c) {
      if (!TB) {
        const int k = k0 + t / BNT + (256 / BNT) * c;
        const int n = n0 + (t % BNT) * 4;
#pragma unroll
        for (int j = 0; j < 4; ++j) rb[4 * c + j] = (k < kend && n + j < N) ? B[(long)k * g.ldb + n + j] : 0.f;
      } else {
        const int n = n0 + t / BKT + (256 / BKT) * c;
        const int k = k0 + (t % BKT) * 4;
#pragma unroll
        for (int j = 0; j < 4; ++j) rb[4 * c + j] = (n < N && k + j < kend) ? B[(long)n * g.ldb + k + j] : 0.f;
      }
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int c = 0; c < LA / 4; ++c)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int mm = !TA ? t / AK + (256 / AK) * c : (t % AM) * 4 + j;
        const int kk = !TA ? (t % AK) * 4 + j : t / AM + (256 / AM) * c;
        split_bf16(ra[4 * c + j], &Ah[mm][kk], &Al[mm][kk]);
      }
#pragma unroll
    for (int c = 0; c < LB / 4; ++c)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int nn = !TB ? (t % BNT) * 4 + j : t / BKT + (256 / BKT) * c;
        const int kk = !TB ? t / BNT + (256 / BNT) * c : (t % BKT) * 4 + j;
        split_bf16(rb[4 * c + j], &Bh[nn][kk], &Bl[nn][kk]);
      }
  };

  f4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  const int lr = lane & 15, lk = lane >> 4;
  if (kbeg < kend) {
    load(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += BK3) {
      __syncthreads();
      stash();
      __syncthreads();
      if (k0 + BK3 < kend) load(k0 + BK3);
      // operand lane l: A(i = l%16, k = 8 (l/16) + v), B(k = 8 (l/16) + v, j = l%16),
      // v = 0..7: the same k for the same (l/16, v) in both operands
      bf8 ah[TM], al[TM], bh[TN], bl[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        ah[i] = __builtin_bit_cast(bf8, *reinterpret_cast<const s8*>(&Ah[wm * WM + i * 16 + lr][8 * lk]));
        al[i] = __builtin_bit_cast(bf8, *reinterpret_cast<const s8*>(&Al[wm * WM + i * 16 + lr][8 * lk]));
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        bh[j] = __builtin_bit_cast(bf8, *reinterpret_cast<const s8*>(&Bh[wn * WN + j * 16 + lr][8 * lk]));
        bl[j] = __builtin_bit_cast(bf8, *reinterpret_cast<const s8*>(&Bl[wn * WN + j * 16 + lr][8 * lk]));
      }
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
        }
    }
  }

  // register r of lane l holds row 4 (l/16) + r, column l%16 of the tile
  if (splitk > 1) {
    double* __restrict__ W = work + (long)ks * M * N;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int col = n0 + wn * WN + j * 16 + lr;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = m0 + wm * WM + i * 16 + 4 * lk + r;
          if (row < M && col < N) W[(long)row * N + col] = (double)acc[i][j][r];
        }
      }
  } else {
    TO* __restrict__ C = static_cast<TO*>(g.C) + b0 * g.sC[0] + b1 * g.sC[1] + b2 * g.sC[2];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int col = n0 + wn * WN + j * 16 + lr;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = m0 + wm * WM + i * 16 + 4 * lk + r;
          if (row < M && col < N) C[(long)row * g.ldc + col] = (TO)acc[i][j][r];
        }
      }
  }
}

template <int BM, int BN, bool TA, bool TB, int TAG, typename TO>
__global__ __launch_bounds__(256) void gemm_bf3_kernel(Gemm g, int splitk, int kchunk, double* work) {
  gemm_bf3_tile<BM, BN, TA, TB, TO>(g, blockIdx.y * BM, blockIdx.x * BN, blockIdx.z, splitk, kchunk, work);
}

template <int BM, int BN, bool TA, bool TB, int TAG, typename TO>
__global__ __launch_bounds__(256) void gemm_bf3_group_kernel(GroupArgs a) {
  int local;
  const int q = group_find<BM, BN>(a, blockIdx.x, &local);
  const GroupItem& it = a.it[q];
  const int tn = local % it.tiles_n, tm = (local / it.tiles_n) % it.tiles_m;
  const int z = local / (it.tiles_n * it.tiles_m);
  gemm_bf3_tile<BM, BN, TA, TB, TO>(it.g, tm * BM, tn * BN, z, it.splitk, it.kchunk, it.work);
}

// Deterministic split-K reduction: C[row*ldc + col] = sum_ks work[ks][row][col].
template <typename TO>
__global__ void splitk_reduce(const double* __restrict__ work, int splitk, int M, int N,
                              TO* __restrict__ C, long ldc) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long MN = (long)M * N;
  if (idx >= MN) return;
  double s = 0.0;
  for (int k = 0; k < splitk; ++k) s += work[k * MN + idx];
  const int row = (int)(idx / N), col = (int)(idx % N);
  C[(long)row * ldc + col] = (TO)s;
}

// The split-K reductions of a grouped launch (problems with splitk > 1;
// `first` counts 256-element blocks here), each in the order of the plain one.
template <typename TO>
__global__ void splitk_reduce_group(GroupArgs a) {
  int local;
  const int q = group_find<1, 1>(a, blockIdx.x, &local);
  const GroupItem& it = a.it[q];
  const long idx = (long)local * blockDim.x + threadIdx.x;
  const long MN = (long)it.g.M * it.g.N;
  if (idx >= MN) return;
  double s = 0.0;
  for (int k = 0; k < it.splitk; ++k) s += it.work[k * MN + idx];
  const int row = (int)(idx / it.g.N), col = (int)(idx % it.g.N);
  static_cast<TO*>(it.g.C)[(long)row * it.g.ldc + col] = (TO)s;
}

namespace {

template <int BM, int BN, int TAG, typename TI, typename TO>
void launch(const Gemm& g, int splitk, int kchunk, double* work, hipStream_t s) {
  dim3 grid((g.N + BN - 1) / BN, (g.M + BM - 1) / BM, g.nb[0] * g.nb[1] * g.nb[2] * splitk);
  dim3 block(256);
  if (!g.transA && !g.transB)
    hipLaunchKernelGGL((gemm_kernel<BM, BN, false, false, TAG, TI, TO>), grid, block, 0, s, g, splitk, kchunk, work);
  else if (g.transA && !g.transB)
    hipLaunchKernelGGL((gemm_kernel<BM, BN, true, false, TAG, TI, TO>), grid, block, 0, s, g, splitk, kchunk, work);
  else if (!g.transA && g.transB)
    hipLaunchKernelGGL((gemm_kernel<BM, BN, false, true, TAG, TI, TO>), grid, block, 0, s, g, splitk, kchunk, work);
  else
    hipLaunchKernelGGL((gemm_kernel<BM, BN, true, true, TAG, TI, TO>), grid, block, 0, s, g, splitk, kchunk, work);
  XTRG_HIP(hipGetLastError());
}

template <int BM, int BN, int TAG, typename TO>
void launch_bf3(const Gemm& g, int splitk, int kchunk, double* work, hipStream_t s) {
  dim3 grid((g.N + BN - 1) / BN, (g.M + BM - 1) / BM, g.nb[0] * g.nb[1] * g.nb[2] * splitk);
  dim3 block(256);
  if (!g.transA && !g.transB)
    hipLaunchKernelGGL((gemm_bf3_kernel<BM, BN, false, false, TAG, TO>), grid, block, 0, s, g, splitk, kchunk, work);
  else if (g.transA && !g.transB)
    hipLaunchKernelGGL((gemm_bf3_kernel<BM, BN, true, false, TAG, TO>), grid, block, 0, s, g, splitk, kchunk, work);
  else if (!g.transA && g.transB)
    hipLaunchKernelGGL((gemm_bf3_kernel<BM, BN, false, true, TAG, TO>), grid, block, 0, s, g, splitk, kchunk, work);
  else
    hipLaunchKernelGGL((gemm_bf3_kernel<BM, BN, true, true, TAG, TO>), grid, block, 0, s, g, splitk, kchunk, work);
  XTRG_HIP(hipGetLastError());
}

template <typename TO>
void launch_bf3_sized(const Gemm& g, bool big, int sk, int kchunk, double* work, hipStream_t s) {
  if (g.tag == 1) {
    if (big) launch_bf3<128, 128, 1, TO>(g, sk, kchunk, work, s);
    else launch_bf3<64, 64, 1, TO>(g, sk, kchunk, work, s);
  } else {
    if (big) launch_bf3<128, 128, 0, TO>(g, sk, kchunk, work, s);
    else launch_bf3<64, 64, 0, TO>(g, sk, kchunk, work, s);
  }
}

template <typename TI, typename TO>
void launch_sized(const Gemm& g, bool big, int sk, int kchunk, double* work, hipStream_t s) {
  if (g.tag == 1) {
    if (big) launch<128, 128, 1, TI, TO>(g, sk, kchunk, work, s);
    else launch<64, 64, 1, TI, TO>(g, sk, kchunk, work, s);
  } else {
    if (big) launch<128, 128, 0, TI, TO>(g, sk, kchunk, work, s);
    else launch<64, 64, 0, TI, TO>(g, sk, kchunk, work, s);
  }
}

int choose_splitk(const Gemm& g, bool big) {
  const long batch = (long)g.nb[0] * g.nb[1] * g.nb[2];
  if (batch != 1) return 1;
  const int bm = big ? 128 : 64, bn = big ? 128 : 64;
  const long tiles = (long)((g.M + bm - 1) / bm) * ((g.N + bn - 1) / bn);
  const long target = 1024;   // workgroups to fill 256 CUs several times over
  if (tiles >= target || g.K < 256) return 1;
  long sk = (target + tiles - 1) / tiles;
  sk = std::min<long>(sk, g.K / 128);
  sk = std::min<long>(sk, 64);
  return (int)std::max<long>(sk, 1);
}

bool use_big(const Gemm& g) { return g.M >= 128 && g.N >= 128; }

// Grouped launches: problems that share a kernel (precision, output type,
// tile size, transposes, tag) go out together, kGroup per launch.
struct Plan {
  bool big;
  int sk, kchunk;
  int key;
};

Plan plan_of(const Gemm& g, bool have_work) {
  Plan p;
  p.big = use_big(g) && !g.tiles64;
  p.sk = choose_splitk(g, p.big);
  if (!have_work || g.K <= 0) p.sk = 1;
  p.kchunk = g.K;
  if (p.sk > 1) {
    p.kchunk = ((g.K + p.sk - 1) / p.sk + BK - 1) / BK * BK;
    p.sk = (g.K + p.kchunk - 1) / p.kchunk;
  }
  const int c64 = g.prec == GEMM_F64 || g.out64;
  p.key = ((((g.prec * 2 + c64) * 2 + p.big) * 2 + g.transA) * 2 + g.transB) * 2 + (g.tag == 1);
  return p;
}

template <int BM, int BN, int TAG, typename TI, typename TO>
void launch_group(const GroupArgs& a, int blocks, int prec, bool tA, bool tB, hipStream_t s) {
  dim3 grid(blocks), block(256);
  if (prec == GEMM_BF16X3) {
    if (!tA && !tB) hipLaunchKernelGGL((gemm_bf3_group_kernel<BM, BN, false, false, TAG, TO>), grid, block, 0, s, a);
    else if (tA && !tB) hipLaunchKernelGGL((gemm_bf3_group_kernel<BM, BN, true, false, TAG, TO>), grid, block, 0, s, a);
    else if (!tA && tB) hipLaunchKernelGGL((gemm_bf3_group_kernel<BM, BN, false, true, TAG, TO>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((gemm_bf3_group_kernel<BM, BN, true, true, TAG, TO>), grid, block, 0, s, a);
  } else {
    if (!tA && !tB) hipLaunchKernelGGL((gemm_group_kernel<BM, BN, false, false, TAG, TI, TO>), grid, block, 0, s, a);
    else if (tA && !tB) hipLaunchKernelGGL((gemm_group_kernel<BM, BN, true, false, TAG, TI, TO>), grid, block, 0, s, a);
    else if (!tA && tB) hipLaunchKernelGGL((gemm_group_kernel<BM, BN, false, true, TAG, TI, TO>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((gemm_group_kernel<BM, BN, true, true, TAG, TI, TO>), grid, block, 0, s, a);
  }
  XTRG_HIP(hipGetLastError());
}

template <typename TI, typename TO>
void launch_group_sized(const GroupArgs& a, int blocks, const Gemm& g0, bool big, hipStream_t s) {
  const bool tA = g0.transA, tB = g0.transB;
  if (g0.tag == 1) {
    if (big) launch_group<128, 128, 1, TI, TO>(a, blocks, g0.prec, tA, tB, s);
    else launch_group<64, 64, 1, TI, TO>(a, blocks, g0.prec, tA, tB, s);
  } else {
    if (big) launch_group<128, 128, 0, TI, TO>(a, blocks, g0.prec, tA, tB, s);
    else launch_group<64, 64, 0, TI, TO>(a, blocks, g0.prec, tA, tB, s);
  }
}

}  // namespace

size_t gemm_grouped_work(const std::vector<Gemm>& gs) {
  size_t w = 0;
  for (const Gemm& g : gs)
    if (g.M > 0 && g.N > 0) w += gemm_splitk_work(g);
  return w;
}

void gemm_grouped(const std::vector<Gemm>& gs, hipStream_t s, double* work, size_t work_cap) {
  const bool have_work = work != nullptr && work_cap >= gemm_grouped_work(gs);
  std::vector<Plan> plans(gs.size());
  for (size_t q = 0; q < gs.size(); ++q) plans[q] = plan_of(gs[q], have_work);
  std::vector<char> done(gs.size(), 0);
  size_t woff = 0;
  for (size_t q0 = 0; q0 < gs.size(); ++q0) {
    if (done[q0] || gs[q0].M <= 0 || gs[q0].N <= 0) continue;
    // every problem of q0's kernel, up to kGroup per launch
    GroupArgs a{};
    int blocks = 0;
    std::vector<size_t> members;
    for (size_t q = q0; q < gs.size() && a.n < kGroup; ++q) {
      const Gemm& g = gs[q];
      if (done[q] || g.M <= 0 || g.N <= 0 || plans[q].key != plans[q0].key) continue;
      done[q] = 1;
      members.push_back(q);
      const Plan& p = plans[q];
      const int bm = p.big ? 128 : 64;
      GroupItem& it = a.it[a.n++];
      it.g = g;
      it.splitk = p.sk;
      it.kchunk = p.kchunk;
      it.work = p.sk > 1 ? work + woff : nullptr;
      if (p.sk > 1) woff += (size_t)p.sk * g.M * g.N;
      it.tiles_n = (g.N + bm - 1) / bm;
      it.tiles_m = (g.M + bm - 1) / bm;
      it.first = blocks;
      blocks += it.tiles_n * it.tiles_m * g.nb[0] * g.nb[1] * g.nb[2] * p.sk;
    }
    const Gemm& g0 = gs[q0];
    const bool big = plans[q0].big;
    const bool c64 = g0.prec == GEMM_F64 || g0.out64;
    if (g0.prec == GEMM_F64) launch_group_sized<double, double>(a, blocks, g0, big, s);
    else if (c64) launch_group_sized<float, double>(a, blocks, g0, big, s);
    else launch_group_sized<float, float>(a, blocks, g0, big, s);
    // the split-K reductions of this launch's problems
    GroupArgs r{};
    int rblocks = 0;
    for (int j = 0; j < a.n; ++j) {
      const GroupItem& it = a.it[j];
      if (it.splitk <= 1) continue;
      GroupItem& ri = r.it[r.n++];
      ri = it;
      ri.first = rblocks;
      rblocks += (int)(((long)it.g.M * it.g.N + 255) / 256);
    }
    if (r.n > 0) {
      if (c64) hipLaunchKernelGGL(splitk_reduce_group<double>, dim3(rblocks), dim3(256), 0, s, r);
      else hipLaunchKernelGGL(splitk_reduce_group<float>, dim3(rblocks), dim3(256), 0, s, r);
      XTRG_HIP(hipGetLastError());
    }
  }
}

size_t gemm_splitk_work(const Gemm& g) {
  const int sk = choose_splitk(g, use_big(g) && !g.tiles64);
  return sk > 1 ? (size_t)sk * g.M * g.N : 0;
}

void gemm(const Gemm& g, hipStream_t s, double* work, size_t work_cap) {
  if (g.M <= 0 || g.N <= 0) return;
  const bool big = use_big(g) && !g.tiles64;
  int sk = choose_splitk(g, big);
  if (sk > 1 && (work == nullptr || work_cap < (size_t)sk * g.M * g.N)) sk = 1;
  if (g.K <= 0) sk = 1;
  int kchunk = g.K;
  if (sk > 1) {
    kchunk = ((g.K + sk - 1) / sk + BK - 1) / BK * BK;
    sk = (g.K + kchunk - 1) / kchunk;
  }
  const bool c64 = g.prec == GEMM_F64 || g.out64;   // FP32 and BF16X3 take float operands
  if (g.prec == GEMM_F64) launch_sized<double, double>(g, big, sk, kchunk, work, s);
  else if (g.prec == GEMM_F32 && c64) launch_sized<float, double>(g, big, sk, kchunk, work, s);
  else if (g.prec == GEMM_F32) launch_sized<float, float>(g, big, sk, kchunk, work, s);
  else if (g.prec == GEMM_BF16X3 && c64) launch_bf3_sized<double>(g, big, sk, kchunk, work, s);
  else if (g.prec == GEMM_BF16X3) launch_bf3_sized<float>(g, big, sk, kchunk, work, s);
  else throw Error(-1, "gemm: unknown precision");
  if (sk > 1) {
    const long MN = (long)g.M * g.N;
    if (c64)
      hipLaunchKernelGGL(splitk_reduce<double>, dim3((MN + 255) / 256), dim3(256), 0, s, work, sk, g.M, g.N,
                         static_cast<double*>(g.C), g.ldc);
    else
      hipLaunchKernelGGL(splitk_reduce<float>, dim3((MN + 255) / 256), dim3(256), 0, s, work, sk, g.M, g.N,
                         static_cast<float*>(g.C), g.ldc);
    XTRG_HIP(hipGetLastError());
  }
}

}  // namespace xtrg
