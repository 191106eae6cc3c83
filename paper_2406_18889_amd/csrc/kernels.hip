// Device kernels of the sliced contraction path, written for gfx950
// (64-wide wavefronts, MFMA matrix cores, LDS).
//
// Complex products on MFMA (Methods C: each step is a pairwise contraction;
// the paper ran it with a vendor einsum or transpose-GEMM, here it is one
// kernel that reads operands in place).  A complex product
// C = sum_k A[m,k] B[n,k] is the real product of A viewed as an m x 2K real
// matrix ((re, im) interleaved, exactly as stored) with a 2N x 2K real
// matrix B' whose rows 2n and 2n+1 are (Br, -Bi) and (Bi, Br) interleaved:
//   row 2n   : sum Ar Br - Ai Bi = Re C
//   row 2n+1 : sum Ar Bi + Ai Br = Im C
// This is the four-real-product form; B' is built in LDS while the tile is
// staged, and the accumulator rows 2n, 2n+1 land in the same lane, so each
// lane writes whole complex numbers.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cstdint>
#include <type_traits>

#include "kernels.h"

namespace lf {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));

constexpr float HALF_MAX = 65504.0f;

template <int NS>
__device__ __forceinline__ int64_t scatter_bits(int64_t v, const int64_t (&st)[NS], int nb) {
  // branch-free, eight bits a round: the eight strides of a round are loaded
  // together (one wait) and masked by their bits; bits of v at or above nb
  // are dropped, so the strides read past nb (inside the array) add nothing.
  // (With a branch per bit, each stride's load from the kernel arguments
  // was waited for on its own: one memory latency per bit of every offset.)
  static_assert(NS % 8 == 0, "whole rounds stay inside the array");
  v &= (int64_t(1) << nb) - 1;
  int64_t s = 0;
  for (int b = 0; b < nb; b += 8) {
#pragma unroll
    for (int i = 0; i < 8; ++i) s += st[b + i] & -((v >> (b + i)) & 1);
  }
  return s;
}

// ------------------------------------------------------------ element io
template <typename T> struct CIO;
template <> struct CIO<float> {
  __device__ static __forceinline__ void load(const float* p, int64_t i, float& re, float& im) {
    float2 v = reinterpret_cast<const float2*>(p)[i];
    re = v.x;
    im = v.y;
  }
  __device__ static __forceinline__ unsigned store(float* p, int64_t i, float re, float im) {
    reinterpret_cast<float2*>(p)[i] = make_float2(re, im);
    return 0;
  }
};
template <> struct CIO<_Float16> {
  __device__ static __forceinline__ void load(const _Float16* p, int64_t i, float& re, float& im) {
    f16x2 v = reinterpret_cast<const f16x2*>(p)[i];
    re = float(v[0]);
    im = float(v[1]);
  }
  // values beyond the half range are clamped to +-HALF_MAX (NaN to 0) and
  // counted; written without branches (a median of three and selects)
  __device__ static __forceinline__ uint32_t pack(float re, float im, unsigned& bad) {
    bad = unsigned(!(fabsf(re) <= HALF_MAX)) | unsigned(!(fabsf(im) <= HALF_MAX));
    re = re != re ? 0.0f : __builtin_amdgcn_fmed3f(re, -HALF_MAX, HALF_MAX);
    im = im != im ? 0.0f : __builtin_amdgcn_fmed3f(im, -HALF_MAX, HALF_MAX);
    f16x2 v;
    v[0] = (_Float16)re;
    v[1] = (_Float16)im;
    uint32_t w;
    __builtin_memcpy(&w, &v, 4);
    return w;
  }
  __device__ static __forceinline__ unsigned store(_Float16* p, int64_t i, float re, float im) {
    unsigned bad;
    reinterpret_cast<uint32_t*>(p)[i] = pack(re, im, bad);
    return bad;
  }
};

// Saturation count (rare, so an atomic only when nonzero) and, when asked
// for, the running maximum of |re|,|im| (one atomic per wave).
__device__ __forceinline__ void block_amax_sat(float local_max, unsigned local_sat, float* amax,
                                               unsigned* sat) {
  if (sat) {
    for (int o = 32; o > 0; o >>= 1) local_sat += __shfl_xor(local_sat, o);
    if ((threadIdx.x & 63) == 0 && local_sat) atomicAdd(sat, local_sat);
  }
  if (amax) {
    for (int o = 32; o > 0; o >>= 1) local_max = fmaxf(local_max, __shfl_xor(local_max, o));
    if ((threadIdx.x & 63) == 0 && local_max > 0.0f)
      atomicMax(reinterpret_cast<unsigned*>(amax), __float_as_uint(local_max));
  }
}

// --------------------------------------------------------------- thin
// One thread per (z, m) row; up to 8 result columns per pass.  Used for
// steps with a narrow side (a large tensor against a gate or small branch),
// which are bound by HBM traffic: every A element is read once, every C
// element written once.
// The body takes the block number and the block count explicitly, so that a
// grouped launch can run several steps' blocks (see gett_thin_group).
template <typename TA, typename TB, typename TO>
__device__ __forceinline__ void thin_body(const GettArgs& a, int64_t blk, int64_t nblk) {
  constexpr int NB = 8;
  const int64_t M = int64_t(1) << a.nm, N = int64_t(1) << a.nn, K = int64_t(1) << a.nk;
  const int64_t rows = (int64_t(1) << a.nz) * M;
  __shared__ int64_t cnT[256];
  for (int n = threadIdx.x; n < N && n < 256; n += blockDim.x) cnT[n] = scatter_bits(n, a.cn, a.nn);
  __syncthreads();
  const TA* A = static_cast<const TA*>(a.A);
  const TB* B = static_cast<const TB*>(a.B);
  TO* C = static_cast<TO*>(a.C);
  float lmax = 0.0f;
  unsigned lsat = 0;
  for (int64_t r = blk * int64_t(blockDim.x) + threadIdx.x; r < rows; r += nblk * blockDim.x) {
    const int64_t z = r >> a.nm, m = r & (M - 1);
    const int64_t cbase = scatter_bits(z, a.cz, a.nz) + scatter_bits(m, a.cm, a.nm);
    const int64_t arow = (a.offA ? a.offA[z] : z * M * K) + m * K;
    const int64_t bz = a.offB ? a.offB[z] : z * N * K;
    for (int64_t n0 = 0; n0 < N; n0 += NB) {
      float cr[NB], ci[NB];
#pragma unroll
      for (int j = 0; j < NB; ++j) { cr[j] = 0.0f; ci[j] = 0.0f; }
      for (int64_t k = 0; k < K; ++k) {
        float ar, ai;
        CIO<TA>::load(A, arow + k, ar, ai);
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          if (n0 + j < N) {
            float br, bi;
            CIO<TB>::load(B, bz + (n0 + j) * K + k, br, bi);
            cr[j] += ar * br - ai * bi;
            ci[j] += ar * bi + ai * br;
          }
        }
      }
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        int64_t n = n0 + j;
        if (n >= N) break;
        float re = cr[j] * a.scale, im = ci[j] * a.scale;
        lmax = fmaxf(lmax, fmaxf(fabsf(re), fabsf(im)));
        if (!a.amax_only) {
          int64_t off = cbase + (n < 256 ? cnT[n] : scatter_bits(n, a.cn, a.nn));
          lsat += CIO<TO>::store(C, off, re, im);
        }
      }
    }
  }
  block_amax_sat(lmax, lsat, a.amax, a.sat);
}

template <typename TA, typename TB, typename TO>
__global__ void __launch_bounds__(256) gett_thin(GettArgs a) {
  thin_body<TA, TB, TO>(a, blockIdx.x, gridDim.x);
}

// Several independent small streaming steps in one launch: block b runs for
// the step whose block range holds it.  A step of a few hundred rows costs
// mostly its launch (a few microseconds each, one after another); grouped,
// the steps' memory latencies overlap and the launch is paid once.
__global__ void __launch_bounds__(256) gett_thin_group(const GroupStep* tab, int n) {
  int64_t b = blockIdx.x;
  int i = 0;
  while (i + 1 < n && b >= tab[i].blocks) {
    b -= tab[i].blocks;
    ++i;
  }
  const GroupStep& g = tab[i];
  switch (g.combo) {
    case 0: thin_body<float, float, float>(g.a, b, g.blocks); break;
    case 1: thin_body<_Float16, float, float>(g.a, b, g.blocks); break;
    case 4: thin_body<float, float, _Float16>(g.a, b, g.blocks); break;
    case 5: thin_body<_Float16, float, _Float16>(g.a, b, g.blocks); break;
    case 3: thin_body<_Float16, _Float16, float>(g.a, b, g.blocks); break;
    case 7: thin_body<_Float16, _Float16, _Float16>(g.a, b, g.blocks); break;
    default: break;
  }
}

int64_t thin_blocks(const GettArgs& a) {
  const int64_t rows = (int64_t(1) << a.nz) << a.nm;
  int64_t blocks = (rows + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  return blocks < 1 ? 1 : blocks;
}

hipError_t launch_thin_group(const GroupStep* tab, int n, int64_t total_blocks, hipStream_t s) {
  if (n < 1 || total_blocks < 1 || total_blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(gett_thin_group, dim3(unsigned(total_blocks)), dim3(256), 0, s, tab, n);
  return hipGetLastError();
}

// ------------------------------------------------------------- narrow
// Steps whose B side is small (N K <= 256 complex) and M >= 256: every
// workgroup lies in one batch entry, stages that entry's B in LDS once, and
// each thread loads its A row (K complex) with vector loads, then forms the
// N results with B read by broadcast from LDS.  HBM traffic is one read of
// A and one write of C.
template <typename T> struct RowLoad;
template <> struct RowLoad<_Float16> {
  template <int K>
  __device__ static __forceinline__ void load(const _Float16* p, float (&re)[K], float (&im)[K]) {
    if constexpr (K >= 4) {
#pragma unroll
      for (int c = 0; c < K / 4; ++c) {
        uint4 v = reinterpret_cast<const uint4*>(p)[c];
        uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          f16x2 h;
          __builtin_memcpy(&h, &w[e], 4);
          re[4 * c + e] = float(h[0]);
          im[4 * c + e] = float(h[1]);
        }
      }
    } else {
#pragma unroll
      for (int e = 0; e < K; ++e) {
        f16x2 h = reinterpret_cast<const f16x2*>(p)[e];
        re[e] = float(h[0]);
        im[e] = float(h[1]);
      }
    }
  }
};
template <> struct RowLoad<float> {
  template <int K>
  __device__ static __forceinline__ void load(const float* p, float (&re)[K], float (&im)[K]) {
    if constexpr (K >= 2) {
#pragma unroll
      for (int c = 0; c < K / 2; ++c) {
        float4 v = reinterpret_cast<const float4*>(p)[c];
        re[2 * c] = v.x;
        im[2 * c] = v.y;
        re[2 * c + 1] = v.z;
        im[2 * c + 1] = v.w;
      }
    } else {
      float2 v = reinterpret_cast<const float2*>(p)[0];
      re[0] = v.x;
      im[0] = v.y;
    }
  }
};

template <typename TA, typename TB, typename TO, int K, int RPT>
__global__ void __launch_bounds__(256) gett_narrow(GettArgs a) {
  __shared__ float2 sB[256];
  __shared__ int64_t cnT[256];
  const int64_t M = int64_t(1) << a.nm;
  const int N = 1 << a.nn;
  // a block takes 256 RPT consecutive rows of one z; thread t takes rows
  // t, t + 256, ..., so that each of its RPT row loads is coalesced across
  // the block and all of them are in flight together
  const int64_t r0 = int64_t(blockIdx.x) * (256 * RPT);
  const int64_t z = r0 >> a.nm;
  const int64_t bz = a.offB ? a.offB[z] : z * N * K;
  const TB* B = static_cast<const TB*>(a.B);
  for (int i = threadIdx.x; i < N * K; i += blockDim.x) {
    float br, bi;
    CIO<TB>::load(B, bz + i, br, bi);
    sB[i] = make_float2(br, bi);
  }
  for (int i = threadIdx.x; i < N; i += blockDim.x) cnT[i] = scatter_bits(i, a.cn, a.nn);
  const int64_t abase = a.offA ? a.offA[z] : z * M * K;
  float ar[RPT][K], ai[RPT][K];
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    const int64_t m = (r0 + threadIdx.x + 256 * j) & (M - 1);
    RowLoad<TA>::template load<K>(static_cast<const TA*>(a.A) + 2 * (abase + m * K), ar[j], ai[j]);
  }
  __syncthreads();
  const int64_t czv = scatter_bits(z, a.cz, a.nz);
  TO* C = static_cast<TO*>(a.C);
  float lmax = 0.0f;
  unsigned lsat = 0;
  // row j of this thread is mb + 256 j + tid (M >= 256 and, with RPT > 1,
  // a multiple of 256 RPT): its low 8 bits are the thread's and the rest
  // is the same in every lane, so that part of its offset is scalar work
  // (mb has no bits below bit 8 + log2 RPT, so 256 j adds its strides bit
  // by bit)
  const int64_t mb = r0 & (M - 1);
  const int64_t lo = scatter_bits(int64_t(threadIdx.x), a.cm, 8);
  const int64_t hi = czv + lo + scatter_bits(mb, a.cm, a.nm);
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    int64_t cbase = hi;
#pragma unroll
    for (int b = 0; (1 << b) < RPT; ++b)
      if ((j >> b) & 1) cbase += a.cm[8 + b];
    for (int n = 0; n < N; ++n) {
      float cr = 0.f, ci = 0.f;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const float2 bv = sB[n * K + k];
        cr += ar[j][k] * bv.x - ai[j][k] * bv.y;
        ci += ar[j][k] * bv.y + ai[j][k] * bv.x;
      }
      cr *= a.scale;
      ci *= a.scale;
      lmax = fmaxf(lmax, fmaxf(fabsf(cr), fabsf(ci)));
      if (!a.amax_only) lsat += CIO<TO>::store(C, cbase + cnT[n], cr, ci);
    }
  }
  block_amax_sat(lmax, lsat, a.amax, a.sat);
}

template <typename TA, typename TB, typename TO, int K>
static hipError_t launch_narrow_k(const GettArgs& a, hipStream_t s) {
  // rows per thread: enough bytes in flight per thread for short rows
  constexpr int RPT = K <= 2 ? 8 : (K <= 4 ? 4 : (K <= 8 ? 2 : 1));
  const int64_t rows = (int64_t(1) << a.nz) << a.nm;
  const dim3 b = dim3(256);
  if ((int64_t(1) << a.nm) >= 256 * RPT) {
    const int64_t blocks = rows / (256 * RPT);
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((gett_narrow<TA, TB, TO, K, RPT>), dim3(unsigned(blocks)), b, 0, s, a);
  } else {
    const int64_t blocks = rows / 256;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((gett_narrow<TA, TB, TO, K, 1>), dim3(unsigned(blocks)), b, 0, s, a);
  }
  return hipGetLastError();
}

template <typename TA, typename TB, typename TO>
static hipError_t launch_narrow(const GettArgs& a, hipStream_t s) {
  switch (a.nk) {
    case 0: return launch_narrow_k<TA, TB, TO, 1>(a, s);
    case 1: return launch_narrow_k<TA, TB, TO, 2>(a, s);
    case 2: return launch_narrow_k<TA, TB, TO, 4>(a, s);
    case 3: return launch_narrow_k<TA, TB, TO, 8>(a, s);
    case 4: return launch_narrow_k<TA, TB, TO, 16>(a, s);
    case 5: return launch_narrow_k<TA, TB, TO, 32>(a, s);
    case 6: return launch_narrow_k<TA, TB, TO, 64>(a, s);
    default: return hipErrorInvalidValue;
  }
}

// --------------------------------------------------------------- MFMA
// Block tile: 128 values of m by 64 complex values of n (128 rows of B'),
// four waves in a 2 x 2 arrangement, each owning 2 x 2 MFMA 32x32 blocks.
// MFMA operand "A" is the expanded B' tile (rows n'), operand "B" is the A
// tile (columns m), so a lane's accumulator rows 2n, 2n+1 are re, im of one
// complex result.
template <typename TI> struct MfmaTraits;
template <> struct MfmaTraits<float> {
  static constexpr int BK = 16;   // complex k per LDS tile
  static constexpr int KS = 2;    // reals per MFMA
  static constexpr int PAD = 4;
};
template <> struct MfmaTraits<_Float16> {
  static constexpr int BK = 32;
  static constexpr int KS = 16;
  static constexpr int PAD = 8;
};

constexpr int MF_BM = 128;
constexpr int MF_BN = 64;

template <typename TI>
__device__ __forceinline__ f32x16 mfma_step(const TI* sB, const TI* sA, int rowB, int rowA, int lda,
                                            int kk, int lane, f32x16 acc);

template <>
__device__ __forceinline__ f32x16 mfma_step<float>(const float* sB, const float* sA, int rowB,
                                                   int rowA, int lda, int kk, int lane, f32x16 acc) {
  float x = sB[rowB * lda + kk + (lane >> 5)];
  float y = sA[rowA * lda + kk + (lane >> 5)];
  return __builtin_amdgcn_mfma_f32_32x32x2f32(x, y, acc, 0, 0, 0);
}

template <>
__device__ __forceinline__ f32x16 mfma_step<_Float16>(const _Float16* sB, const _Float16* sA,
                                                      int rowB, int rowA, int lda, int kk, int lane,
                                                      f32x16 acc) {
  f16x8 x = *reinterpret_cast<const f16x8*>(&sB[rowB * lda + kk + 8 * (lane >> 5)]);
  f16x8 y = *reinterpret_cast<const f16x8*>(&sA[rowA * lda + kk + 8 * (lane >> 5)]);
  return __builtin_amdgcn_mfma_f32_32x32x16_f16(x, y, acc, 0, 0, 0);
}

// 16-byte chunk of CPC complex values
template <typename TI> struct Chunk {
  static constexpr int CPC = 16 / (2 * int(sizeof(TI)));
};

template <typename TI, typename TO>
__global__ void __launch_bounds__(256) gett_mfma(GettArgs a) {
  using Tr = MfmaTraits<TI>;
  constexpr int BK = Tr::BK, BK2 = 2 * BK, LDA = BK2 + Tr::PAD;
  constexpr int CPC = Chunk<TI>::CPC;          // complex per 16 B
  constexpr int CH_ROW = BK / CPC;             // 16 B chunks per tile row
  __shared__ __attribute__((aligned(16))) TI sA[MF_BM * LDA];
  __shared__ __attribute__((aligned(16))) TI sB[2 * MF_BN * LDA];
  __shared__ int64_t cmT[MF_BM];
  __shared__ int64_t cnT[MF_BN];

  const int64_t M = int64_t(1) << a.nm, N = int64_t(1) << a.nn, K = int64_t(1) << a.nk;
  const int64_t mt = (M + MF_BM - 1) / MF_BM, nt = (N + MF_BN - 1) / MF_BN;
  int64_t bid = blockIdx.x;
  const int64_t tn = bid % nt;
  bid /= nt;
  const int64_t tm = bid % mt;
  const int64_t z = bid / mt;
  const int64_t m0 = tm * MF_BM, n0 = tn * MF_BN;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wn = w & 1, wm = w >> 1;
  const int validM = int(M - m0 < MF_BM ? M - m0 : MF_BM);
  const int validN = int(N - n0 < MF_BN ? N - n0 : MF_BN);

  for (int i = tid; i < MF_BM; i += 256) cmT[i] = scatter_bits(m0 + i, a.cm, a.nm);
  for (int i = tid; i < MF_BN; i += 256) cnT[i] = scatter_bits(n0 + i, a.cn, a.nn);
  const int64_t czv = scatter_bits(z, a.cz, a.nz);

  const TI* Ab = static_cast<const TI*>(a.A) + 2 * ((a.offA ? a.offA[z] : z * M * K) + m0 * K);
  const TI* Bb = static_cast<const TI*>(a.B) + 2 * ((a.offB ? a.offB[z] : z * N * K) + n0 * K);

  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;

  // MODE 0: whole tiles and K a multiple of BK, no bounds tests.  MODE 1: K
  // a multiple of the 16-byte chunk, so that every chunk lies wholly inside
  // or wholly outside the operand: one outside reads row 0, chunk 0 and is
  // zeroed by a mask, and no load sits behind a branch (a predicated load
  // merges its value after the branch, and the compiler then waits for
  // every load before issuing the next).  MODE 2: K below one chunk,
  // element by element.
  // one K step: each thread's A chunks (NA) and B chunks (NB).  The loads
  // of step k + 1 are issued into registers before the MFMAs of step k and
  // stored to LDS after them, so that their latency overlaps the MFMAs and
  // the loads of one step overlap each other.
  constexpr int NA = MF_BM * CH_ROW / 256, NB = MF_BN * CH_ROW / 256;
  static_assert(NA * 256 == MF_BM * CH_ROW && NB * 256 == MF_BN * CH_ROW, "chunks per thread");
  auto put_b = [&](int r, int ch, const TI* re, const TI* im) __attribute__((always_inline)) {
    TI row0[2 * CPC], row1[2 * CPC];
#pragma unroll
    for (int e = 0; e < CPC; ++e) {
      row0[2 * e] = re[e];
      row0[2 * e + 1] = -im[e];
      row1[2 * e] = im[e];
      row1[2 * e + 1] = re[e];
    }
    *reinterpret_cast<float4*>(&sB[(2 * r) * LDA + 2 * ch * CPC]) = *reinterpret_cast<float4*>(row0);
    *reinterpret_cast<float4*>(&sB[(2 * r + 1) * LDA + 2 * ch * CPC]) = *reinterpret_cast<float4*>(row1);
  };
  auto main_loop = [&](auto mode_tag) {
    constexpr int MODE = decltype(mode_tag)::value;
    // raw chunks of the next step and, in MODE 1, which of them lie inside
    // (bit i: A chunk i, bit NA + i: B chunk i); the mask is applied when
    // the chunk is stored, so that nothing waits for the loads before then
    typedef uint32_t v4u __attribute__((ext_vector_type(4)));
    v4u va[NA], vb[NB];
    uint32_t okm = ~0u;
    auto load_step = [&](int64_t k0) __attribute__((always_inline)) {
      if constexpr (MODE == 1) okm = 0u;
#pragma unroll
      for (int i = 0; i < NA; ++i) {
        const int c = tid + 256 * i, r = c / CH_ROW, ch = c % CH_ROW;
        const int64_t kc = k0 + int64_t(ch) * CPC;
        if constexpr (MODE == 0) {
          va[i] = *reinterpret_cast<const v4u*>(Ab + 2 * (int64_t(r) * K + kc));
        } else {
          const bool ok = r < validM && kc < K;
          va[i] = *reinterpret_cast<const v4u*>(Ab + 2 * (int64_t(ok ? r : 0) * K + (ok ? kc : 0)));
          okm |= uint32_t(ok) << i;
        }
      }
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        const int c = tid + 256 * i, r = c / CH_ROW, ch = c % CH_ROW;
        const int64_t kc = k0 + int64_t(ch) * CPC;
        if constexpr (MODE == 0) {
          vb[i] = *reinterpret_cast<const v4u*>(Bb + 2 * (int64_t(r) * K + kc));
        } else {
          const bool ok = r < validN && kc < K;
          vb[i] = *reinterpret_cast<const v4u*>(Bb + 2 * (int64_t(ok ? r : 0) * K + (ok ? kc : 0)));
          okm |= uint32_t(ok) << (NA + i);
        }
      }
    };
    auto keep = [&](v4u x, int bit) __attribute__((always_inline)) {
      if constexpr (MODE == 0) return x;
      return x & (0u - ((okm >> bit) & 1u));
    };
    if constexpr (MODE < 2) load_step(0);
    for (int64_t k0 = 0; k0 < K; k0 += BK) {
      if constexpr (MODE < 2) {
#pragma unroll
        for (int i = 0; i < NA; ++i) {
          const int c = tid + 256 * i, r = c / CH_ROW, ch = c % CH_ROW;
          *reinterpret_cast<v4u*>(&sA[r * LDA + 2 * ch * CPC]) = keep(va[i], i);
        }
#pragma unroll
        for (int i = 0; i < NB; ++i) {
          const int c = tid + 256 * i, r = c / CH_ROW, ch = c % CH_ROW;
          const v4u x = keep(vb[i], NA + i);
          TI tmp[2 * CPC], re[CPC], im[CPC];
          __builtin_memcpy(tmp, &x, 16);
#pragma unroll
          for (int e = 0; e < CPC; ++e) { re[e] = tmp[2 * e]; im[e] = tmp[2 * e + 1]; }
          put_b(r, ch, re, im);
        }
      } else {
        // K below one chunk: element by element
        for (int c = tid; c < MF_BM * CH_ROW; c += 256) {
          const int r = c / CH_ROW, ch = c % CH_ROW;
          const int64_t kc = k0 + int64_t(ch) * CPC;
          TI* dst = &sA[r * LDA + 2 * ch * CPC];
#pragma unroll
          for (int e = 0; e < CPC; ++e) {
            const bool ok = r < validM && kc + e < K;
            dst[2 * e] = ok ? Ab[2 * (int64_t(r) * K + kc + e)] : TI(0);
            dst[2 * e + 1] = ok ? Ab[2 * (int64_t(r) * K + kc + e) + 1] : TI(0);
          }
        }
        for (int c = tid; c < MF_BN * CH_ROW; c += 256) {
          const int r = c / CH_ROW, ch = c % CH_ROW;
          const int64_t kc = k0 + int64_t(ch) * CPC;
          TI re[CPC], im[CPC];
#pragma unroll
          for (int e = 0; e < CPC; ++e) {
            const bool ok = r < validN && kc + e < K;
            re[e] = ok ? Bb[2 * (int64_t(r) * K + kc + e)] : TI(0);
            im[e] = ok ? Bb[2 * (int64_t(r) * K + kc + e) + 1] : TI(0);
          }
          put_b(r, ch, re, im);
        }
      }
      __syncthreads();
      if constexpr (MODE < 2)
        if (k0 + BK < K) load_step(k0 + BK);
#pragma unroll
      for (int kk = 0; kk < BK2; kk += Tr::KS) {
#pragma unroll
        for (int bn = 0; bn < 2; ++bn)
#pragma unroll
          for (int bm = 0; bm < 2; ++bm)
            acc[bn][bm] = mfma_step<TI>(sB, sA, wn * 64 + bn * 32 + (lane & 31),
                                        wm * 64 + bm * 32 + (lane & 31), LDA, kk, lane, acc[bn][bm]);
      }
      __syncthreads();
    }
  };
  if (validM == MF_BM && validN == MF_BN && K % BK == 0)
    main_loop(std::integral_constant<int, 0>{});
  else if (K % CPC == 0)
    main_loop(std::integral_constant<int, 1>{});
  else
    main_loop(std::integral_constant<int, 2>{});

  // epilogue: lane holds column m, rows n' = 8(v/4) + 4(lane/32) + v%4
  TO* C = static_cast<TO*>(a.C);
  float lmax = 0.0f;
  unsigned lsat = 0;
#pragma unroll
  for (int bn = 0; bn < 2; ++bn)
#pragma unroll
    for (int bm = 0; bm < 2; ++bm) {
      const int ml = wm * 64 + bm * 32 + (lane & 31);
      if (ml >= validM) continue;
      const int64_t cb = czv + cmT[ml];
#pragma unroll
      for (int v = 0; v < 16; v += 2) {
        const int np = wn * 64 + bn * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        const int nl = np >> 1;
        if (nl >= validN) continue;
        const float re = acc[bn][bm][v] * a.scale, im = acc[bn][bm][v + 1] * a.scale;
        lmax = fmaxf(lmax, fmaxf(fabsf(re), fabsf(im)));
        if (!a.amax_only) lsat += CIO<TO>::store(C, cb + cnT[nl], re, im);
      }
    }
  block_amax_sat(lmax, lsat, a.amax, a.sat);
}

// ------------------------------------------------ MFMA, large f16 tiles
// Complex-half operands.  Four waves in 2 (m) x 2 (n) arrangement; each wave
// owns WM x WN MFMA 32x32x16 blocks (32 WM values of m by 32 WN rows of B',
// i.e. 16 WN complex n), so the block tile is 64 WM (m) x 32 WN (complex n)
// x 32 (complex k).  Both LDS tiles hold plain (re, im) rows; the B'
// fragment of a lane is formed in registers from 4 complex values of row
// n = n'/2: row 2n gets (Br, -Bi), row 2n+1 gets (Bi, Br).  The next K tile
// is fetched from HBM into registers while the current one is multiplied.
//
// ST = 1: one LDS buffer, two barriers per K step.  ST = 2: two LDS
// buffers; tile t+1 is written to the idle buffer after tile t's MFMAs were
// issued, one barrier per K step.  (A third stage needs a second register
// set of prefetched chunks, which does not fit beside the 4 x 4 accumulators
// without spilling.)  A K step of BK = 64 (one buffer) doubles
// the MFMA work that covers the HBM latency of the next step's loads, which
// the register budget beside a 4 x 4 wave tile allows only once.
//
// Tile order (ORDER): 0 numbers tiles n fastest, then m, then z;
// 1 gives each XCD a contiguous range of tiles in groups of 8 m-tiles.
// With order 0 every XCD touches every A panel (HBM reads of A up to 8x);
// order 1 reads A once and B once per group, but measured 5% slower on fat,
// compute-bound steps, so the autotuner picks per step shape.
//
// FULL (chosen at launch: M, N multiples of the block tile and K of the K
// step, so every tile is whole) drops the bounds tests from the loads: a
// predicated load merges its value after a branch, and the compiler then
// waits for every load before issuing the next, which serialises the HBM
// latency of a whole K step.
// LDS row of a tile with BK complex k: 2 BK halves and a 16 B pad, so that
// the rows read by one fragment load start in distinct bank groups
template <int BK> struct BigK {
  static constexpr int LDK = 2 * BK + 8;   // halves per LDS row
  static constexpr int CPR = BK / 4;       // 16 B chunks per row
};

// B' fragment from 4 complex values (re, im halves per 32-bit word): for
// even rows n' the word becomes (re, -im), for odd rows (im, re).  Done with
// one byte permutation and one xor per word, the selector and sign mask
// chosen per lane once (a per-lane ternary here compiles to branches).
struct BPrime {
  uint32_t sel, xm;
  __device__ __forceinline__ explicit BPrime(int parity)
      : sel(parity ? 0x01000302u : 0x03020100u), xm(parity ? 0u : 0x80000000u) {}
};

__device__ __forceinline__ f16x8 bprime_frag(uint4 raw, const BPrime& bp) {
  uint32_t w[4] = {raw.x, raw.y, raw.z, raw.w};
#pragma unroll
  for (int i = 0; i < 4; ++i) w[i] = __builtin_amdgcn_perm(w[i], w[i], bp.sel) ^ bp.xm;
  f16x8 r;
  __builtin_memcpy(&r, w, 16);
  return r;
}

template <int WM, int WN> struct BigTile {
  static constexpr int BM = 64 * WM;   // m per block
  static constexpr int BN = 32 * WN;   // complex n per block
};

__device__ __forceinline__ void big_tile_of(int64_t bid, int64_t nblk, int order, int64_t mt, int64_t nt,
                                            int64_t& z, int64_t& tm, int64_t& tn) {
  if (order == 0) {
    tn = bid % nt;
    bid /= nt;
    tm = bid % mt;
    z = bid / mt;
    return;
  }
  // blocks are dealt to the 8 XCDs round-robin: give each XCD a contiguous
  // range of tiles, walked in groups of 8 m-tiles that sweep n together
  if ((nblk & 7) == 0) bid = (bid & 7) * (nblk >> 3) + (bid >> 3);
  const int64_t per_z = mt * nt;
  z = bid / per_z;
  const int64_t r = bid - z * per_z;
  const int64_t per_group = 8 * nt, g = r / per_group, rg = r - g * per_group;
  const int64_t first = g * 8, gsz = mt - first < 8 ? mt - first : 8;
  tm = first + rg % gsz;
  tn = rg / gsz;
}

template <typename TO, int WM, int WN, int MINB, int ST, int BK, bool FULL, int ORDER>
__global__ void __launch_bounds__(256, MINB) gett_mfma_big(GettArgs a) {
  constexpr int BM = BigTile<WM, WN>::BM, BN = BigTile<WM, WN>::BN;
  constexpr int BG_BK = BK, BG_LDK = BigK<BK>::LDK, CPR = BigK<BK>::CPR;
  constexpr int NA = BM * CPR / 256, NB = BN * CPR / 256;   // 16 B chunks per thread
  constexpr int NBUF = ST >= 2 ? 2 : 1;
  static_assert(ST == 1 || ST == 2, "stages");
  // one LDS block: the operand tiles during the K loop, then (whole
  // complex-half tiles) the result tile, staged for an ordered write-out
  constexpr bool STAGE = FULL && std::is_same<TO, _Float16>::value;
  constexpr int SROW = BN + 1;   // staged row (words): odd, so lanes of consecutive m hit distinct banks
  constexpr int MAIN_BYTES = NBUF * (BM + BN) * BG_LDK * 2;
  constexpr int STAGE_BYTES = STAGE ? BM * SROW * 4 : 0;
  constexpr int SMEM = MAIN_BYTES > STAGE_BYTES ? MAIN_BYTES : STAGE_BYTES;
  __shared__ __attribute__((aligned(16))) unsigned char smem[SMEM];
  typedef _Float16 TileA[BM * BG_LDK];
  typedef _Float16 TileB[BN * BG_LDK];
  TileA* sA = reinterpret_cast<TileA*>(smem);
  TileB* sB = reinterpret_cast<TileB*>(smem + NBUF * BM * BG_LDK * 2);
  __shared__ int64_t cmT[BM];
  __shared__ int64_t cnT[BN];

  const int64_t M = int64_t(1) << a.nm, N = int64_t(1) << a.nn, K = int64_t(1) << a.nk;
  const int64_t mt = (M + BM - 1) / BM, nt = (N + BN - 1) / BN;
  int64_t z, tm, tn;
  big_tile_of(blockIdx.x, gridDim.x, ORDER, mt, nt, z, tm, tn);
  const int64_t m0 = tm * BM, n0 = tn * BN;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w & 1, wn = w >> 1;
  const int validM = int(M - m0 < BM ? M - m0 : BM);
  const int validN = int(N - n0 < BN ? N - n0 : BN);
  for (int i = tid; i < BM; i += 256) cmT[i] = scatter_bits(m0 + i, a.cm, a.nm);
  for (int i = tid; i < BN; i += 256) cnT[i] = scatter_bits(n0 + i, a.cn, a.nn);
  const int64_t czv = scatter_bits(z, a.cz, a.nz);
  const _Float16* Ab = static_cast<const _Float16*>(a.A) + 2 * ((a.offA ? a.offA[z] : z * M * K) + m0 * K);
  const _Float16* Bb = static_cast<const _Float16*>(a.B) + 2 * ((a.offB ? a.offB[z] : z * N * K) + n0 * K);

  f32x16 acc[WN][WM];
#pragma unroll
  for (int i = 0; i < WN; ++i)
#pragma unroll
    for (int j = 0; j < WM; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;

  // one 16 B chunk = 4 complex; a tile row of BK complex = CPR chunks
  {
    auto fetch = [&](const _Float16* base, int valid, int row, int ch, int64_t k0) -> uint4 {
      const int64_t kc = k0 + 4 * ch;
      if constexpr (FULL) {
        (void)valid;
        return *reinterpret_cast<const uint4*>(base + 2 * (int64_t(row) * K + kc));
      } else {
        uint4 v = make_uint4(0, 0, 0, 0);
        if (row < valid) {
          const _Float16* p = base + 2 * (int64_t(row) * K + kc);
          if (kc + 4 <= K) {
            v = *reinterpret_cast<const uint4*>(p);
          } else if (kc < K) {
            uint32_t t[4] = {0, 0, 0, 0};
            for (int e = 0; e < 4 && kc + e < K; ++e) t[e] = reinterpret_cast<const uint32_t*>(p)[e];
            v = make_uint4(t[0], t[1], t[2], t[3]);
          }
        }
        return v;
      }
    };
    auto load = [&](uint4 (&ra)[NA], uint4 (&rb)[NB], int64_t k0) {
#pragma unroll
      for (int i = 0; i < NA; ++i) {
        const int c = tid + 256 * i;
        ra[i] = fetch(Ab, validM, c / CPR, c % CPR, k0);
      }
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        const int c = tid + 256 * i;
        rb[i] = fetch(Bb, validN, c / CPR, c % CPR, k0);
      }
    };
    auto store = [&](const uint4 (&ra)[NA], const uint4 (&rb)[NB], int buf) {
#pragma unroll
      for (int i = 0; i < NA; ++i) {
        const int c = tid + 256 * i;
        *reinterpret_cast<uint4*>(&sA[buf][(c / CPR) * BG_LDK + 8 * (c % CPR)]) = ra[i];
      }
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        const int c = tid + 256 * i;
        *reinterpret_cast<uint4*>(&sB[buf][(c / CPR) * BG_LDK + 8 * (c % CPR)]) = rb[i];
      }
    };
    const BPrime bp(lane & 1);   // parity of the B' row n' of this lane
    // k steps [kk0, kk1) of the tile in LDS buffer buf
    auto compute_part = [&](int buf, int kk0, int kk1) {
      const _Float16* cA = sA[buf];
      const _Float16* cB = sB[buf];
#pragma unroll
      for (int kk = kk0; kk < kk1; kk += 8) {
        const int koff = 2 * (kk + 4 * (lane >> 5));   // halves
        f16x8 af[WM], bf[WN];
#pragma unroll
        for (int bm = 0; bm < WM; ++bm)
          af[bm] = *reinterpret_cast<const f16x8*>(&cA[(wm * 32 * WM + bm * 32 + (lane & 31)) * BG_LDK + koff]);
#pragma unroll
        for (int bn = 0; bn < WN; ++bn) {
          const int np = wn * 32 * WN + bn * 32 + (lane & 31);
          uint4 raw = *reinterpret_cast<const uint4*>(&cB[(np >> 1) * BG_LDK + koff]);
          bf[bn] = bprime_frag(raw, bp);
        }
#pragma unroll
        for (int bn = 0; bn < WN; ++bn)
#pragma unroll
          for (int bm = 0; bm < WM; ++bm)
            acc[bn][bm] = __builtin_amdgcn_mfma_f32_32x32x16_f16(bf[bn], af[bm], acc[bn][bm], 0, 0, 0);
      }
    };
    auto compute = [&](int buf) { compute_part(buf, 0, BG_BK); };
    const int64_t T = (K + BG_BK - 1) / BG_BK;
    uint4 ra0[NA], rb0[NB];
    if constexpr (ST == 2) {
      load(ra0, rb0, 0);
      store(ra0, rb0, 0);
      __syncthreads();
      for (int64_t t = 0; t < T; ++t) {
        const int cur = int(t & 1);
        if (t + 1 < T) load(ra0, rb0, (t + 1) * BG_BK);
        // the writes of tile t+1 into the other buffer (last read before the
        // previous barrier) go out before the last k step of tile t, so the
        // LDS writes overlap that step's MFMAs
        compute_part(cur, 0, BG_BK - 8);
        if (t + 1 < T) store(ra0, rb0, cur ^ 1);
        compute_part(cur, BG_BK - 8, BG_BK);
        __syncthreads();
      }
    } else {
      load(ra0, rb0, 0);
      for (int64_t t = 0; t < T; ++t) {
        store(ra0, rb0, 0);
        __syncthreads();
        if (t + 1 < T) load(ra0, rb0, (t + 1) * BG_BK);
        compute(0);
        __syncthreads();
      }
    }
  }

  TO* C = static_cast<TO*>(a.C);
  float lmax = 0.0f;
  unsigned lsat = 0;
  if constexpr (STAGE) {
    // Whole complex-half tile: results go to LDS as (re, im) half pairs, then
    // leave in the order of the output's strides.  The tile's element index
    // e has one bit per tile bit of m (8) and of n (log2 BN), sorted by the
    // output stride of that bit; consecutive threads take consecutive e, so
    // the smallest strides run across lanes and the stores coalesce however
    // the consumer laid the result out.
    constexpr int LM = 8, LN = BN == 128 ? 7 : (BN == 64 ? 6 : 5), LT = LM + LN;
    constexpr int PER = (BM * BN) / 256;   // elements per thread
    uint32_t* stage = reinterpret_cast<uint32_t*>(smem);
    if (a.amax_only) {
      // calibration pass: the running maximum only, nothing is stored
#pragma unroll
      for (int bn = 0; bn < WN; ++bn)
#pragma unroll
        for (int bm = 0; bm < WM; ++bm)
#pragma unroll
          for (int v = 0; v < 16; ++v) lmax = fmaxf(lmax, fabsf(acc[bn][bm][v] * a.scale));
      block_amax_sat(lmax, 0u, a.amax, a.sat);
      return;
    }
    __shared__ int64_t sStv[LT];   // the tile's bit strides in ascending order (stable)
    __shared__ int sBit[LT];       // and which tile bit each is (0..LM-1 m, LM.. n)
    if (tid < LT) {
      // rank of bit tid among the LT strides: one thread per bit instead of
      // a sort in every thread
      const int64_t v = tid < LM ? a.cm[tid] : a.cn[tid - LM];
      int r = 0;
#pragma unroll
      for (int j = 0; j < LT; ++j) {
        const int64_t u = j < LM ? a.cm[j] : a.cn[j - LM];
        r += (u < v) || (u == v && j < tid);
      }
      sStv[r] = v;
      sBit[r] = tid;
    }
    __syncthreads();   // every wave is done with the operand tiles
#pragma unroll
    for (int bn = 0; bn < WN; ++bn)
#pragma unroll
      for (int bm = 0; bm < WM; ++bm) {
        const int ml = wm * 32 * WM + bm * 32 + (lane & 31);
#pragma unroll
        for (int v = 0; v < 16; v += 2) {
          const int nl = (wn * 32 * WN + bn * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3)) >> 1;
          float re = acc[bn][bm][v] * a.scale, im = acc[bn][bm][v + 1] * a.scale;
          lsat += unsigned(!(fabsf(re) <= HALF_MAX)) + unsigned(!(fabsf(im) <= HALF_MAX));
          re = re != re ? 0.0f : __builtin_amdgcn_fmed3f(re, -HALF_MAX, HALF_MAX);
          im = im != im ? 0.0f : __builtin_amdgcn_fmed3f(im, -HALF_MAX, HALF_MAX);
          f16x2 h;
          h[0] = (_Float16)re;
          h[1] = (_Float16)im;
          uint32_t wv;
          __builtin_memcpy(&wv, &h, 4);
          stage[ml * SROW + nl] = wv;
        }
      }
    // element e = tid + 256 j: its low 8 bits come from tid, the rest from j
    auto split = [&](int e, int lo, int hi, int64_t& addr, int& idx) {
      addr = 0;
      int ml = 0, nl = 0;
#pragma unroll
      for (int i = lo; i < hi; ++i)
        if ((e >> (i - lo)) & 1) {
          addr += sStv[i];
          const int b = sBit[i];
          if (b < LM) ml |= 1 << b;
          else nl |= 1 << (b - LM);
        }
      idx = ml * SROW + nl;
    };
    int64_t loAddr;
    int loIdx;
    split(tid, 0, 8, loAddr, loIdx);
    // address and staging offsets of the high sorted bits (taken from j),
    // the same in every thread: scalar registers
    constexpr int HB = LT - 8;
    static_assert((1 << HB) == PER, "high bits enumerate the thread's elements");
    int64_t hS[HB];
    int hI[HB];
#pragma unroll
    for (int b = 0; b < HB; ++b) {
      const int64_t v = sStv[8 + b];
      hS[b] = (int64_t(__builtin_amdgcn_readfirstlane(int(v >> 32))) << 32) |
              uint32_t(__builtin_amdgcn_readfirstlane(int(v)));
      const int bb = __builtin_amdgcn_readfirstlane(sBit[8 + b]);
      hI[b] = bb < LM ? (1 << bb) * SROW : (1 << (bb - LM));
    }
    __syncthreads();
    if (!a.amax_only) {
      const int64_t base = czv + cmT[0] + cnT[0] + loAddr;
      uint32_t* Cw = reinterpret_cast<uint32_t*>(C);
      // element j of this thread: offsets built from element j with its
      // lowest set bit cleared (one scalar add each); streaming stores: the
      // tile is written once and read by a later step
      int64_t ad[PER];
      int ix[PER];
      ad[0] = 0;
      ix[0] = 0;
#pragma unroll
      for (int j = 0; j < PER; ++j) {
        if (j > 0) {
          const int b = __builtin_ctz(j);
          ad[j] = ad[j & (j - 1)] + hS[b];
          ix[j] = ix[j & (j - 1)] + hI[b];
        }
        __builtin_nontemporal_store(stage[loIdx + ix[j]], &Cw[base + ad[j]]);
      }
    }
  } else {
#pragma unroll
  for (int bn = 0; bn < WN; ++bn)
#pragma unroll
    for (int bm = 0; bm < WM; ++bm) {
      const int ml = wm * 32 * WM + bm * 32 + (lane & 31);
      if (ml >= validM) continue;
      const int64_t cb = czv + cmT[ml];
#pragma unroll
      for (int v = 0; v < 16; v += 2) {
        const int np = wn * 32 * WN + bn * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        const int nl = np >> 1;
        if (nl >= validN) continue;
        const float re = acc[bn][bm][v] * a.scale, im = acc[bn][bm][v + 1] * a.scale;
        lmax = fmaxf(lmax, fmaxf(fabsf(re), fabsf(im)));
        if (!a.amax_only) lsat += CIO<TO>::store(C, cb + cnT[nl], re, im);
      }
    }
  }
  block_amax_sat(lmax, lsat, a.amax, a.sat);
}

// ------------------------------------------------------------ DMA-fed MFMA
// The 256 m x 128 n complex tile, run by eight waves (two per SIMD, each
// 128 m x 32 n, the accumulators in 128 VGPRs) so that one wave's MFMAs
// cover the other's LDS waits, or by four (one per SIMD, 128 m x 64 n, the
// accumulators in AGPRs).  The real and imaginary parts of C are separate
// 32 x 32 MFMA blocks that share the A fragment: each lane reads one whole
// B row chunk, and both operand forms of it, (Br, -Bi) and (Bi, Br), are
// made in registers (one operation per 32-bit word), so no two lanes read
// the same LDS bytes.  Whole tiles only (M % 256, N % 128, K % 32 == 0,
// chosen on the host).  The operand tiles reach LDS without passing through
// registers: each global->LDS load writes 64 lanes x 16 B = 1 KB at the LDS
// address held in M0, three stages deep.  Rows are not padded (the 1 KB
// lands contiguously); chunk c (16 B) of row r sits at slot c ^ ((r >> 1) & 7),
// which keeps each fragment read free of bank conflicts.  The loads are
// issued from inline assembly: the compiler's own form of this load makes it
// wait for every outstanding load before any LDS access.  Here the waits are
// explicit (see the main loop).
constexpr int DMA_BM = 256, DMA_BN = 128, DMA_BK = 32;   // default tile (the m side may be 128)

typedef __attribute__((address_space(3))) void* lds_void_ptr;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// one 1 KB global->LDS load: lane L's 16 B from sbase + voff go to LDS
// address m0 + 16 L (sbase and m0 wave-uniform)
__device__ __forceinline__ void dma_load16(uint32_t voff, const void* sbase, uint32_t m0) {
  asm volatile("s_nop 0\n\tglobal_load_lds_dwordx4 %0, %1" ::"v"(voff), "s"(sbase), "{m0}"(m0) : "memory");
}

// s_waitcnt vmcnt(N) lgkmcnt(0), then s_barrier (N: this wave's loads that
// may still be in flight)
template <int N>
__device__ __forceinline__ void wait_loads_barrier() {
  static_assert(N == 0 || N == 2 || N == 6 || N == 8 || N == 12 || N == 15, "vmcnt immediate");
  if constexpr (N == 0) asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory");
  if constexpr (N == 2) asm volatile("s_waitcnt vmcnt(2) lgkmcnt(0)\n\ts_barrier" ::: "memory");
  if constexpr (N == 6) asm volatile("s_waitcnt vmcnt(6) lgkmcnt(0)\n\ts_barrier" ::: "memory");
  if constexpr (N == 8) asm volatile("s_waitcnt vmcnt(8) lgkmcnt(0)\n\ts_barrier" ::: "memory");
  if constexpr (N == 12) asm volatile("s_waitcnt vmcnt(12) lgkmcnt(0)\n\ts_barrier" ::: "memory");
  if constexpr (N == 15) asm volatile("s_waitcnt vmcnt(15) lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// NW = 8: eight waves (two per SIMD), each 128 m x 32 n, 8 MFMAs per k step,
// 128 accumulator registers.  NW = 4: four waves (one per SIMD), each 128 m x
// 64 n, 16 MFMAs per k step, 256 accumulator registers (AGPRs): fewer LDS
// bytes and VALU operations per MFMA, and the waits must be hidden by the
// order of one wave's instructions alone.
//
// BM = 128, STAGES = 2 (kernels 16 and 17): the 128 m x 128 n tile on four
// waves (each 128 m x 32 n, as in the eight-wave form) with two operand
// stages, so that its LDS (68 KB) lets two workgroups share a CU: one
// workgroup's first loads and write-out run while the other computes, which
// pays on steps with a short K where those fixed costs are a large share.
// With two stages the loads of tile t+1 are issued during tile t and waited
// for before its last k step (the co-resident workgroup covers that wait).
template <typename TO, int ORDER, int NW, int BM = DMA_BM, int STAGES = 3>
__global__ void __launch_bounds__(64 * NW, STAGES == 2 ? 2 : 1) gett_mfma_dma(GettArgs a) {
  static_assert(NW == 4 || NW == 8, "wave count");
  static_assert((BM == 256 && STAGES == 3) || (BM == 128 && STAGES == 2 && NW == 4), "tile forms");
  constexpr int NT = 64 * NW;
  // waves along m (the rest along n): eight waves as 2 x 4 and the 128-row
  // tile's four as 1 x 4, each 128 m x 32 n, so that a wave forms the B'
  // operands of one 32-row block of B per k step for its 8 MFMAs (one VALU
  // operation per MFMA instead of two, for one more LDS read); the 256-row
  // tile's four waves as 2 x 2
  constexpr int MW = (NW == 4 && BM == 128) ? 1 : 2;
  constexpr int WM = BM / (32 * MW), WN = DMA_BN / (32 * (NW / MW));   // 32 x 32 MFMA tiles per wave
  constexpr int SA = BM * 128;                   // bytes of the A tile of a stage
  constexpr int STAGE = (BM + DMA_BN) * 128;     // bytes per stage
  constexpr int A_LOADS = BM * 128 / 1024 / NW, B_LOADS = DMA_BN * 128 / 1024 / NW;
  constexpr int LOADS = A_LOADS + B_LOADS;       // per wave per stage
  constexpr int CHUNK = (LOADS + 3) / 4;         // loads of a tile issued per k step
  static_assert(WM * 32 * MW == BM && LOADS * NW * 1024 == STAGE, "wave grid and loads");
  // operand stages, reused for the staged result tile at the end
  constexpr int SMEM = (STAGES * STAGE > BM * (DMA_BN + 1) * 4 ? STAGES * STAGE : BM * (DMA_BN + 1) * 4);
  __shared__ __attribute__((aligned(1024))) unsigned char smem[(SMEM + 1023) / 1024 * 1024];
  __shared__ int64_t cmT[BM];
  __shared__ int64_t cnT[DMA_BN];

  const int64_t M = int64_t(1) << a.nm, N = int64_t(1) << a.nn, K = int64_t(1) << a.nk;
  const int64_t mt = M / BM, nt = N / DMA_BN;
  int64_t z, tm, tn;
  big_tile_of(blockIdx.x, gridDim.x, ORDER, mt, nt, z, tm, tn);
  const int64_t m0 = tm * BM, n0 = tn * DMA_BN;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = w % MW, wn = w / MW;
  for (int i = tid; i < BM; i += NT) cmT[i] = scatter_bits(m0 + i, a.cm, a.nm);
  for (int i = tid; i < DMA_BN; i += NT) cnT[i] = scatter_bits(n0 + i, a.cn, a.nn);
  const int64_t czv = scatter_bits(z, a.cz, a.nz);
  const unsigned char* Ab =
      static_cast<const unsigned char*>(a.A) + 4 * ((a.offA ? a.offA[z] : z * M * K) + m0 * K);
  const unsigned char* Bb =
      static_cast<const unsigned char*>(a.B) + 4 * ((a.offB ? a.offB[z] : z * N * K) + n0 * K);

  // load i of this wave covers rows 8 (wave's first load + i) .. +7; lane L
  // fills slot L % 8 of row L / 8 of them, i.e. fetches chunk slot ^ swizzle
  uint32_t voA[A_LOADS], voB[B_LOADS];
#pragma unroll
  for (int i = 0; i < A_LOADS; ++i) {
    const int row = (w * A_LOADS + i) * 8 + (lane >> 3), c = (lane & 7) ^ ((row >> 1) & 7);
    voA[i] = uint32_t(row) * uint32_t(K) * 4u + uint32_t(c) * 16u;
  }
#pragma unroll
  for (int i = 0; i < B_LOADS; ++i) {
    const int row = (w * B_LOADS + i) * 8 + (lane >> 3), c = (lane & 7) ^ ((row >> 1) & 7);
    voB[i] = uint32_t(row) * uint32_t(K) * 4u + uint32_t(c) * 16u;
  }
  const uint32_t lds0 = static_cast<uint32_t>(reinterpret_cast<uintptr_t>((lds_void_ptr)smem));
  // group G (0..3) of this wave's loads of tile t into stage st: loads
  // G*CHUNK .. (G+1)*CHUNK-1, the A loads first
  auto issue_group = [&](auto G, int st, int64_t t) __attribute__((always_inline)) {
    constexpr int g = decltype(G)::value;
    const unsigned char* ga = Ab + t * (DMA_BK * 4);
    const unsigned char* gb = Bb + t * (DMA_BK * 4);
    const uint32_t base = lds0 + uint32_t(st) * STAGE;
#pragma unroll
    for (int i = g * CHUNK; i < (g + 1) * CHUNK && i < LOADS; ++i) {
      if (i < A_LOADS) dma_load16(voA[i < A_LOADS ? i : 0], ga, base + uint32_t(w * A_LOADS + i) * 1024u);
      else
        dma_load16(voB[i < A_LOADS ? 0 : i - A_LOADS], gb,
                   base + SA + uint32_t(w * B_LOADS + i - A_LOADS) * 1024u);
    }
  };
  using I0 = std::integral_constant<int, 0>;
  using I1 = std::integral_constant<int, 1>;
  using I2 = std::integral_constant<int, 2>;
  using I3 = std::integral_constant<int, 3>;

  int offA[WM], swA[WM], offB[WN], swB[WN];
#pragma unroll
  for (int bm = 0; bm < WM; ++bm) {
    const int r = wm * 32 * WM + bm * 32 + (lane & 31);
    offA[bm] = r * 128;
    swA[bm] = (r >> 1) & 7;
  }
#pragma unroll
  for (int bn = 0; bn < WN; ++bn) {
    const int r = wn * 32 * WN + bn * 32 + (lane & 31);
    offB[bn] = SA + r * 128;
    swB[bn] = (r >> 1) & 7;
  }
  f16x8 af[2][WM];
  u32x4 rb[2][WN];
  auto frags = [&](const unsigned char* s, int kk, int sl) __attribute__((always_inline)) {
    const int c = (kk >> 2) + (lane >> 5);   // 16 B chunk: 4 complex
    // B first: its B' operands are formed before this A set is needed
#pragma unroll
    for (int bn = 0; bn < WN; ++bn) rb[sl][bn] = *reinterpret_cast<const u32x4*>(s + offB[bn] + ((c ^ swB[bn]) << 4));
#pragma unroll
    for (int bm = 0; bm < WM; ++bm) af[sl][bm] = *reinterpret_cast<const f16x8*>(s + offA[bm] + ((c ^ swA[bm]) << 4));
  };
  // acc[bn][0][bm]: real parts, acc[bn][1][bm]: imaginary parts of the
  // 32 n x 32 m block (bn, bm)
  f32x16 acc[WN][2][WM];
#pragma unroll
  for (int i = 0; i < WN; ++i)
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int j = 0; j < WM; ++j)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[i][p][j][v] = 0.0f;
  // the matrix part of a k step.  With A's rows as (re, im) pairs along k,
  // Re C[n, m] = sum_k A[m, k] . (Br, -Bi)[n, k] and
  // Im C[n, m] = sum_k A[m, k] . (Bi, Br)[n, k]: one B row read from LDS
  // gives both operand rows, by a sign flip of the high half and by a swap
  // of the halves of each 32-bit word.  Then 8 MFMAs.
  auto bprime = [&](auto CS, f16x8 (*bf)[2]) __attribute__((always_inline)) {
    constexpr int cs = decltype(CS)::value;
#pragma unroll
    for (int bn = 0; bn < WN; ++bn) {
      u32x4 re, im;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint32_t x = rb[cs][bn][i];
        re[i] = x ^ 0x80000000u;
        im[i] = __builtin_amdgcn_alignbit(x, x, 16);
      }
      bf[bn][0] = __builtin_bit_cast(f16x8, re);
      bf[bn][1] = __builtin_bit_cast(f16x8, im);
    }
  };
  auto mma = [&](auto CS, f16x8 (*bf)[2]) __attribute__((always_inline)) {
    constexpr int cs = decltype(CS)::value;
#pragma unroll
    for (int bn = 0; bn < WN; ++bn)
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int bm = 0; bm < WM; ++bm)
          acc[bn][p][bm] = __builtin_amdgcn_mfma_f32_32x32x16_f16(bf[bn][p], af[cs][bm], acc[bn][p][bm], 0, 0, 0);
  };
  // One k step: the fragments of the next k step (raw B first, then A) are
  // read into register set NCS while the MFMAs of this step run on set CS
  // and the B' operands bf, and the B' operands of the next step (bfn) are
  // formed from the raw B read at its start.  The scheduling groups issue
  // these one by one between MFMAs, so that the matrix pipe is fed while the
  // reads and the VALU work proceed.
  auto kstep = [&](auto CS, f16x8 (*bf)[2], f16x8 (*bfn)[2], const unsigned char* rs, int rkk)
      __attribute__((always_inline)) {
    constexpr int ncs = decltype(CS)::value ^ 1;
    using NCS = std::integral_constant<int, ncs>;
    frags(rs, rkk, ncs);
    mma(CS, bf);
    bprime(NCS{}, bfn);
    constexpr int READS = WM + WN, MFMAS = 2 * WM * WN;
#pragma unroll
    for (int i = 0; i < READS; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // one LDS read
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // one MFMA
    }
    constexpr int REST = MFMAS - READS, SPREAD = REST >= 8 ? 8 : REST;
    if constexpr (REST > SPREAD) __builtin_amdgcn_sched_group_barrier(0x008, REST - SPREAD, 0);
#pragma unroll
    for (int i = 0; i < SPREAD; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x002, 16 / SPREAD, 0);   // B' VALU
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
    }
    // formed in this step (else the compiler sinks it past the next branch)
#pragma unroll
    for (int bn = 0; bn < WN; ++bn) asm volatile("" : "+v"(bfn[bn][0]), "+v"(bfn[bn][1]));
  };
  static_assert(DMA_BK == 32, "four k steps per tile");
  // Pipeline.  Tile t+3 is requested into the stage of tile t once every wave
  // has passed the barrier in the last k step of tile t (by then all
  // fragments of tile t are in registers); its loads are spread over that k
  // step and the first three of the next tile, a quarter each.  The barrier
  // falls between MFMAs of the same tile and each load has about two tiles of
  // compute to arrive.  Branches (the loads of tiles past the end, the wait
  // count) sit between the k steps, so that each k step is one scheduling
  // region.
  const int64_t T = K / DMA_BK;
  issue_group(I0{}, 0, 0);
  issue_group(I1{}, 0, 0);
  issue_group(I2{}, 0, 0);
  issue_group(I3{}, 0, 0);
  if constexpr (STAGES == 3) {
    if (T > 1) {
      issue_group(I0{}, 1, 1);
      issue_group(I1{}, 1, 1);
      issue_group(I2{}, 1, 1);
      issue_group(I3{}, 1, 1);
    }
    if (T > 2) issue_group(I0{}, 2, 2);
    // tile 0 has landed: only tile 1 and the first group of tile 2 may be in flight
    if (T > 2) wait_loads_barrier<LOADS + CHUNK>();
    else if (T > 1) wait_loads_barrier<LOADS>();
    else wait_loads_barrier<0>();
  } else {
    if (T > 1) issue_group(I0{}, 1, 1);
    // tile 0 has landed: only the first group of tile 1 may be in flight
    if (T > 1) wait_loads_barrier<CHUNK>();
    else wait_loads_barrier<0>();
  }
  frags(smem, 0, 0);
  f16x8 bfe[WN][2], bfo[WN][2];   // B' operands of even and odd k steps
  bprime(I0{}, bfe);
  int st = 0;
  for (int64_t t = 0; t + 1 < T; ++t) {
    const unsigned char* s = smem + st * STAGE;
    if constexpr (STAGES == 3) {
      const int nst = st == 2 ? 0 : st + 1, pst = st == 0 ? 2 : st - 1;   // stages of t+1, t+2
      const bool more = t + 2 < T;
      if (more) issue_group(I1{}, pst, t + 2);
      __builtin_amdgcn_sched_barrier(0);
      kstep(I0{}, bfe, bfo, s, 8);
      __builtin_amdgcn_sched_barrier(0);
      if (more) issue_group(I2{}, pst, t + 2);
      __builtin_amdgcn_sched_barrier(0);
      kstep(I1{}, bfo, bfe, s, 16);
      __builtin_amdgcn_sched_barrier(0);
      if (more) issue_group(I3{}, pst, t + 2);
      __builtin_amdgcn_sched_barrier(0);
      kstep(I0{}, bfe, bfo, s, 24);
      __builtin_amdgcn_sched_barrier(0);
      // tile t+1 has landed (only tile t+2's loads may be in flight) and every
      // wave's reads of tile t have returned: stage st is free
      if (more) wait_loads_barrier<LOADS>();
      else wait_loads_barrier<0>();
      if (t + 3 < T) issue_group(I0{}, st, t + 3);
      __builtin_amdgcn_sched_barrier(0);
      kstep(I1{}, bfo, bfe, smem + nst * STAGE, 0);
      __builtin_amdgcn_sched_barrier(0);
      st = nst;
    } else {
      // tile t+1 goes into the other stage during the first three k steps of
      // tile t (its first group was issued before); tile t+2 into this stage
      // once every wave has passed the barrier before the last k step
      const int nst = st ^ 1;
      issue_group(I1{}, nst, t + 1);
      __builtin_amdgcn_sched_barrier(0);
      kstep(I0{}, bfe, bfo, s, 8);
      __builtin_amdgcn_sched_barrier(0);
      issue_group(I2{}, nst, t + 1);
      __builtin_amdgcn_sched_barrier(0);
      kstep(I1{}, bfo, bfe, s, 16);
      __builtin_amdgcn_sched_barrier(0);
      issue_group(I3{}, nst, t + 1);
      __builtin_amdgcn_sched_barrier(0);
      kstep(I0{}, bfe, bfo, s, 24);
      __builtin_amdgcn_sched_barrier(0);
      // tile t+1 has landed and every wave's reads of tile t have returned
      wait_loads_barrier<0>();
      if (t + 2 < T) issue_group(I0{}, st, t + 2);
      __builtin_amdgcn_sched_barrier(0);
      kstep(I1{}, bfo, bfe, smem + nst * STAGE, 0);
      __builtin_amdgcn_sched_barrier(0);
      st = nst;
    }
  }
  {
    const unsigned char* s = smem + st * STAGE;
    kstep(I0{}, bfe, bfo, s, 8);
    kstep(I1{}, bfo, bfe, s, 16);
    kstep(I0{}, bfe, bfo, s, 24);
    mma(I1{}, bfo);
  }

  TO* C = static_cast<TO*>(a.C);
  float lmax = 0.0f;
  unsigned lsat = 0;
  if constexpr (std::is_same<TO, _Float16>::value) {
    // staged write-out in the order of the output's strides (as in the
    // large kernels): NT threads, PER elements each
    constexpr int BN = DMA_BN, SROW = BN + 1, LM = BM == 256 ? 8 : 7, LN = 7, LT = LM + LN;
    constexpr int LO = NW == 8 ? 9 : 8, PER = (BM * BN) / NT;
    static_assert((1 << LO) == NT && PER <= NT, "thread bits of the write-out");
    static_assert(BM * SROW * 4 <= int(sizeof(smem)), "staged tile fits the operand stages");
    uint32_t* stage = reinterpret_cast<uint32_t*>(smem);
    if (a.amax_only) {
      // calibration pass: the running maximum only, nothing is stored
#pragma unroll
      for (int bn = 0; bn < WN; ++bn)
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
          for (int bm = 0; bm < WM; ++bm)
#pragma unroll
            for (int v = 0; v < 16; ++v) lmax = fmaxf(lmax, fabsf(acc[bn][p][bm][v] * a.scale));
      block_amax_sat(lmax, 0u, a.amax, a.sat);
      return;
    }
    __shared__ int64_t sStv[LT];   // the tile's bit strides in ascending order (stable)
    __shared__ int sBit[LT];       // and which tile bit each is
    if (tid < LT) {
      // rank of bit tid among the LT strides: one thread per bit instead of
      // a sort in every thread
      const int64_t v = tid < LM ? a.cm[tid] : a.cn[tid - LM];
      int r = 0;
#pragma unroll
      for (int j = 0; j < LT; ++j) {
        const int64_t u = j < LM ? a.cm[j] : a.cn[j - LM];
        r += (u < v) || (u == v && j < tid);
      }
      sStv[r] = v;
      sBit[r] = tid;
    }
    __syncthreads();   // every wave is done with the operand tiles
#pragma unroll
    for (int bn = 0; bn < WN; ++bn)
#pragma unroll
      for (int bm = 0; bm < WM; ++bm) {
        const int ml = wm * 32 * WM + bm * 32 + (lane & 31);
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int nl = wn * 32 * WN + bn * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
          float re = acc[bn][0][bm][v] * a.scale, im = acc[bn][1][bm][v] * a.scale;
          lsat += unsigned(!(fabsf(re) <= HALF_MAX)) + unsigned(!(fabsf(im) <= HALF_MAX));
          re = re != re ? 0.0f : __builtin_amdgcn_fmed3f(re, -HALF_MAX, HALF_MAX);
          im = im != im ? 0.0f : __builtin_amdgcn_fmed3f(im, -HALF_MAX, HALF_MAX);
          f16x2 h;
          h[0] = (_Float16)re;
          h[1] = (_Float16)im;
          uint32_t wv;
          __builtin_memcpy(&wv, &h, 4);
          stage[ml * SROW + nl] = wv;
        }
      }
    // element e = tid + NT j: its low LO bits come from tid, the rest from j
    auto split = [&](int e, int lo, int hi, int64_t& addr, int& idx) {
      addr = 0;
      int ml = 0, nl = 0;
#pragma unroll
      for (int i = lo; i < hi; ++i)
        if ((e >> (i - lo)) & 1) {
          addr += sStv[i];
          const int b = sBit[i];
          if (b < LM) ml |= 1 << b;
          else nl |= 1 << (b - LM);
        }
      idx = ml * SROW + nl;
    };
    int64_t loAddr;
    int loIdx;
    split(tid, 0, LO, loAddr, loIdx);
    // address and staging offsets of the high sorted bits (taken from j),
    // the same in every thread: scalar registers
    constexpr int HB = LT - LO;
    static_assert((1 << HB) == PER, "high bits enumerate the thread's elements");
    int64_t hS[HB];
    int hI[HB];
#pragma unroll
    for (int b = 0; b < HB; ++b) {
      const int64_t v = sStv[LO + b];
      hS[b] = (int64_t(__builtin_amdgcn_readfirstlane(int(v >> 32))) << 32) |
              uint32_t(__builtin_amdgcn_readfirstlane(int(v)));
      const int bb = __builtin_amdgcn_readfirstlane(sBit[LO + b]);
      hI[b] = bb < LM ? (1 << bb) * SROW : (1 << (bb - LM));
    }
    __syncthreads();
    if (!a.amax_only) {
      const int64_t base = czv + cmT[0] + cnT[0] + loAddr;
      uint32_t* Cw = reinterpret_cast<uint32_t*>(C);
      // element j of this thread: offsets built from element j with its
      // lowest set bit cleared (one scalar add each); streaming stores: the
      // tile is written once and read by a later step
      int64_t ad[PER];
      int ix[PER];
      ad[0] = 0;
      ix[0] = 0;
#pragma unroll
      for (int j = 0; j < PER; ++j) {
        if (j > 0) {
          const int b = __builtin_ctz(j);
          ad[j] = ad[j & (j - 1)] + hS[b];
          ix[j] = ix[j & (j - 1)] + hI[b];
        }
        __builtin_nontemporal_store(stage[loIdx + ix[j]], &Cw[base + ad[j]]);
      }
    }
  } else {
#pragma unroll
    for (int bn = 0; bn < WN; ++bn)
#pragma unroll
      for (int bm = 0; bm < WM; ++bm) {
        const int ml = wm * 32 * WM + bm * 32 + (lane & 31);
        const int64_t cb = czv + cmT[ml];
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int nl = wn * 32 * WN + bn * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
          const float re = acc[bn][0][bm][v] * a.scale, im = acc[bn][1][bm][v] * a.scale;
          lmax = fmaxf(lmax, fmaxf(fabsf(re), fabsf(im)));
          if (!a.amax_only) lsat += CIO<TO>::store(C, cb + cnT[nl], re, im);
        }
      }
  }
  block_amax_sat(lmax, lsat, a.amax, a.sat);
}

// ------------------------------------------------------------ skinny MFMA
// Steps with a short side: N <= 32 complex (NF = 1 or 2 fragments of 32 B'
// rows), 4 <= K <= 64, complex-half A, M >= 32 GPW.  Each wave multiplies 32
// rows of A at a time by the whole of B', which it holds in registers, with
// MFMA 32x32x16 and no LDS.  A is streamed from HBM once and C written once,
// so the step is bound by HBM rather than by the vector ALU rate of the
// one-row-per-thread kernels; with M = 32 (GPW = 1) it is the batched
// 32 x 32 products of the last stem steps, one wave per batch entry instead
// of a mostly empty tile per entry.  A complex64 B is split into a high and
// a low half (two MFMAs per k step), which keeps its rounding at about 2^-22
// relative.  A wave takes GPW consecutive 32-row groups (its slab of m) of
// ZC consecutive batch entries z, one entry after another: it reloads the A
// (B) fragments only when the gathered block of A (B) changes from one entry
// to the next, so in a batch sorted by the closed bits of a gathered operand
// each of its blocks is read once per run of entries that share it instead
// of once per entry.
template <typename TB, typename TO, int KC, int GPW, int NF = 1, int ZC = 1, int NSB = 0, int PACK = 1, int STG = 0>
__global__ void __launch_bounds__(256) gett_skinny(GettArgs a, int64_t n_waves) {
  constexpr int S = KC >= 8 ? KC / 8 : 1;   // k steps of 16 reals
  constexpr bool SPLIT = std::is_same<TB, float>::value;
  constexpr int BW = SPLIT ? 2 : 1;          // raw 16-byte words of B per (fragment, k step)
  static_assert(NF == 1 || (NF == 2 && !SPLIT), "two B' fragments: complex-half B only");
  static_assert(ZC >= 1 && ZC <= 64, "entries per wave: one lane each for their offsets");
  static_assert(NSB == 0 || (!SPLIT && NF == 1 && NSB <= 16), "staged B: complex-half, one fragment");
  static_assert(PACK == 1 || (NSB > 0 && ZC % PACK == 0), "packed entries read B from the staged copy");
  static_assert(STG == 0 || (GPW == 1 && NF == 2 && PACK == 1 && std::is_same<TO, _Float16>::value),
                "staged write-out: one 32 x 32 complex-half block per entry");
  // STG: each entry's 32 x 32 result is one contiguous 4 KB block of C
  // (checked at launch); the wave writes it to LDS at its place in the block
  // (word o at o ^ 4 ((o >> 6) & 15), so the scattered writes of a wave fall
  // in distinct banks) and copies it out in 16-byte pieces, four store
  // instructions of 1 KB each instead of 16 scattered ones
  __shared__ uint32_t stg[STG ? 4 * 1024 : 1];
  constexpr int RW = KC >= 4 ? KC / 4 + 1 : 2;   // 16-byte words per staged B row (one of padding)
  __shared__ int64_t cnT[16 * NF];
  __shared__ uint4 sB[NSB > 0 ? ZC * NSB * RW : 1];
  const int64_t M = int64_t(1) << a.nm;
  const int64_t Z = int64_t(1) << a.nz;
  const int N = 1 << a.nn;
  const int lane = threadIdx.x & 63;
  if (threadIdx.x < N) cnT[threadIdx.x] = scatter_bits(threadIdx.x, a.cn, a.nn);
  const int slab_bits = a.nm - (GPW == 1 ? 5 : GPW == 2 ? 6 : 7);   // slabs of 32 GPW rows per entry
  if constexpr (NSB > 0) {
    // the four waves of the block share one chunk of ZC entries (at least
    // four slabs, checked at launch): their B blocks are read once, by all
    // threads at a time, into LDS, rather than entry by entry by each wave
    const int CPE = N * (KC / 4);                  // 16-byte words per entry
    const int64_t zc0 = ((int64_t(blockIdx.x) * 4) >> slab_bits) * ZC;
    for (int i = threadIdx.x; i < ZC * CPE; i += 256) {
      const int e = i / CPE, w = i - e * CPE, n = w / (KC / 4), c4 = w - n * (KC / 4);
      const int64_t z = zc0 + e;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (z < Z) {
        const int64_t bz = a.offB ? a.offB[z] : z * int64_t(N) * KC;
        v = *reinterpret_cast<const uint4*>(static_cast<const _Float16*>(a.B) + 2 * (bz + int64_t(n) * KC + 4 * c4));
      }
      sB[(e * NSB + n) * RW + c4] = v;
    }
  }
  __syncthreads();
  const int64_t wave = int64_t(blockIdx.x) * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (wave >= n_waves) return;
  const int64_t m0 = (wave & ((int64_t(1) << slab_bits) - 1)) * (32 * GPW);
  const int64_t z0 = (wave >> slab_bits) * ZC;
  const int kq = 4 * (lane >> 5);                  // complex k offset of this lane in a step
  const BPrime bp(lane & 1);                       // B' row n' = lane % 32 of fragment f: n = 16 f + n' / 2
  const _Float16* Abase = static_cast<const _Float16*>(a.A);
  TO* C = static_cast<TO*>(a.C);
  // the operand offsets of the wave's entries, lane i holding those of entry
  // z0 + i, read once (a gather table lookup per entry would put one memory
  // latency between consecutive entries)
  const int64_t zl = z0 + (lane < ZC ? lane : 0);
  const int64_t myA = zl < Z ? (a.offA ? a.offA[zl] : zl * M * KC) : 0;
  const int64_t myB = zl < Z ? (a.offB ? a.offB[zl] : zl * int64_t(N) * KC) : 0;
  auto lane64 = [](int64_t v, int i) {
    return int64_t((uint64_t(uint32_t(__builtin_amdgcn_readlane(int(uint64_t(v) >> 32), i))) << 32) |
                   uint32_t(__builtin_amdgcn_readlane(int(v), i)));
  };
  auto offA = [&](int64_t z) { return lane64(myA, int(z - z0)); };
  auto offB = [&](int64_t z) { return lane64(myB, int(z - z0)); };
  // result offsets: of the entries (one lane each, as above) and of this
  // lane's rows, which are the same for every entry
  const int64_t myC = scatter_bits(zl, a.cz, a.nz);
  int64_t cbm[GPW];
#pragma unroll
  for (int g = 0; g < GPW; ++g) cbm[g] = scatter_bits(m0 + g * 32 + (lane & 31), a.cm, a.nm);
  // raw B words of an entry (complex-half: 8 halves; complex64: 8 floats in two words)
  auto load_b = [&](int64_t bz, uint4 (&rb)[NF][S][BW]) __attribute__((always_inline)) {
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
      for (int st = 0; st < S; ++st) {
        const int n = 16 * f + ((lane & 31) >> 1);
        const int kc = st * 8 + kq;
#pragma unroll
        for (int w = 0; w < BW; ++w) rb[f][st][w] = make_uint4(0, 0, 0, 0);
        if (n < N && kc < KC) {
          if constexpr (SPLIT) {
            const uint4* p = reinterpret_cast<const uint4*>(static_cast<const float*>(a.B) + 2 * (bz + int64_t(n) * KC + kc));
            rb[f][st][0] = p[0];
            rb[f][st][BW - 1] = p[1];
          } else {
            rb[f][st][0] = *reinterpret_cast<const uint4*>(static_cast<const _Float16*>(a.B) +
                                                           2 * (bz + int64_t(n) * KC + kc));
          }
        }
      }
  };
  // the same from the staged copy (entry e of the chunk)
  auto load_b_lds = [&](int e, uint4 (&rb)[NF][S][BW]) __attribute__((always_inline)) {
#pragma unroll
    for (int st = 0; st < S; ++st) {
      const int n = (lane & 31) >> 1;
      const int kc = st * 8 + kq;
      rb[0][st][0] = (n < N && kc < KC) ? sB[(e * NSB + n) * RW + kc / 4] : make_uint4(0, 0, 0, 0);
    }
  };
  auto load_a = [&](int64_t az, f16x8 (&af)[GPW][S]) __attribute__((always_inline)) {
    const _Float16* A = Abase + 2 * az;
#pragma unroll
    for (int g = 0; g < GPW; ++g)
#pragma unroll
      for (int st = 0; st < S; ++st) {
        const int kc = st * 8 + kq;
        const int64_t m = m0 + g * 32 + (lane & 31);
        if (kc < KC) {
          af[g][st] = *reinterpret_cast<const f16x8*>(A + 2 * (m * KC + kc));
        } else {
#pragma unroll
          for (int e = 0; e < 8; ++e) af[g][st][e] = (_Float16)0.0f;
        }
      }
  };
  // B' fragments from the raw words (complex64: rounded high part and the
  // rounded remainder)
  f16x8 bh[NF][S], bl[S];
  auto form_b = [&](const uint4 (&rb)[NF][S][BW]) __attribute__((always_inline)) {
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
      for (int st = 0; st < S; ++st) {
        if constexpr (SPLIT) {
          float x[8];
          __builtin_memcpy(x, &rb[f][st][0], 16);
          __builtin_memcpy(x + 4, &rb[f][st][BW - 1], 16);
          uint32_t wh[4], wl[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            f16x2 h, l;
            h[0] = (_Float16)x[2 * e];
            h[1] = (_Float16)x[2 * e + 1];
            l[0] = (_Float16)(x[2 * e] - float(h[0]));
            l[1] = (_Float16)(x[2 * e + 1] - float(h[1]));
            __builtin_memcpy(&wh[e], &h, 4);
            __builtin_memcpy(&wl[e], &l, 4);
          }
          bh[f][st] = bprime_frag(make_uint4(wh[0], wh[1], wh[2], wh[3]), bp);
          bl[st] = bprime_frag(make_uint4(wl[0], wl[1], wl[2], wl[3]), bp);
        } else {
          bh[f][st] = bprime_frag(rb[f][st][0], bp);
        }
      }
  };
  // One entry after another; the next entry's B words (and, for one-group
  // waves, its A fragments when its block differs) are requested before this
  // entry's MFMAs, so their latency overlaps the arithmetic and the stores.
  // Waves of several groups reload A in place, only where the block changes.
  constexpr bool PIPE_A = GPW == 1;
  // calibration pass: the running maximum only; otherwise store (the
  // maximum is not needed then)
  const bool store_all = !a.amax_only;
  uint4 rb[NF][S][BW];
  f16x8 af[GPW][S], an[GPW][S];
  float lmax = 0.0f;
  unsigned lsat = 0;
  if constexpr (PACK > 1) {
    // N <= 8: PACK = 16 / N consecutive entries that share their A block go
    // through one B' fragment together (entry j of the pack in B' rows
    // 2N j .. 2N j + 2N - 1), so the MFMAs and the B' operand work of a pack
    // cost what one entry's did.  A pack whose entries differ in A is done
    // entry by entry.
    auto shfl64 = [](int64_t v, int src) {
      return int64_t((uint64_t(uint32_t(__shfl(int(uint64_t(v) >> 32), src))) << 32) |
                     uint32_t(__shfl(int(v), src)));
    };
    auto emit = [&](int g, const f32x16& acc, int e_fixed) __attribute__((always_inline)) {
#pragma unroll
      for (int v = 0; v < 16; v += 2) {
        const int np = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        int e, nl;
        if (e_fixed >= 0) {
          e = e_fixed;
          nl = np >> 1;
          if (4 * (v >> 2) >= N) break;   // no result row in this row group (all lanes)
        } else {
          e = np / (2 * N);
          nl = (np % (2 * N)) >> 1;
        }
        const float re = acc[v] * a.scale, im = acc[v + 1] * a.scale;
        if (nl < N) {
          const int64_t cz = e_fixed >= 0 ? lane64(myC, e) : shfl64(myC, e);
          if (store_all) lsat += CIO<TO>::store(C, cz + cbm[g] + cnT[nl], re, im);
          else lmax = fmaxf(lmax, fmaxf(fabsf(re), fabsf(im)));
        }
      }
    };
    if (z0 < Z) {
      int64_t curA = -1;
      const int np = lane & 31;
      for (int p = 0; p < ZC / PACK; ++p) {
        const int e0 = p * PACK;
        const int64_t a0 = offA(z0 + e0);
        bool same = true;
#pragma unroll
        for (int j = 1; j < PACK; ++j) same = same && offA(z0 + e0 + j) == a0;
        if (same) {
          if (a0 != curA) {
            load_a(a0, af);
            curA = a0;
          }
          const int je = np / (2 * N), nr = (np % (2 * N)) >> 1;
          f16x8 bpk[S];
#pragma unroll
          for (int st = 0; st < S; ++st) {
            const int kc = st * 8 + kq;
            bpk[st] = bprime_frag(kc < KC ? sB[((e0 + je) * NSB + nr) * RW + kc / 4] : make_uint4(0, 0, 0, 0), bp);
          }
#pragma unroll
          for (int g = 0; g < GPW; ++g) {
            f32x16 acc;
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
#pragma unroll
            for (int st = 0; st < S; ++st) acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(bpk[st], af[g][st], acc, 0, 0, 0);
            emit(g, acc, -1);
          }
        } else {
          for (int j = 0; j < PACK; ++j) {
            const int e = e0 + j;
            const int64_t ae = offA(z0 + e);
            if (ae != curA) {
              load_a(ae, af);
              curA = ae;
            }
            load_b_lds(e, rb);
            form_b(rb);
#pragma unroll
            for (int g = 0; g < GPW; ++g) {
              f32x16 acc;
#pragma unroll
              for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
#pragma unroll
              for (int st = 0; st < S; ++st) acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(bh[0][st], af[g][st], acc, 0, 0, 0);
              emit(g, acc, e);
            }
          }
        }
      }
    }
    block_amax_sat(lmax, lsat, a.amax, a.sat);
    return;
  }
  if (z0 < Z) {
    int64_t curB = offB(z0), curA = offA(z0);
    if constexpr (NSB > 0) load_b_lds(0, rb);
    else load_b(curB, rb);
    load_a(curA, af);
    for (int zi = 0; zi < ZC; ++zi) {
      const int64_t z = z0 + zi;
      if (z >= Z) break;
      form_b(rb);
      const bool more = zi + 1 < ZC && z + 1 < Z;
      const int64_t nB = more ? offB(z + 1) : curB;
      const int64_t nA = more ? offA(z + 1) : curA;
      if (nB != curB) {
        if constexpr (NSB > 0) load_b_lds(zi + 1, rb);
        else load_b(nB, rb);
      }
      if constexpr (PIPE_A) {
        if (nA != curA) load_a(nA, an);
      }
      const int64_t czv = lane64(myC, zi);
#pragma unroll
      for (int g = 0; g < GPW; ++g) {
        f32x16 acc[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
          for (int v = 0; v < 16; ++v) acc[f][v] = 0.0f;
#pragma unroll
        for (int st = 0; st < S; ++st)
#pragma unroll
          for (int f = 0; f < NF; ++f) {
            acc[f] = __builtin_amdgcn_mfma_f32_32x32x16_f16(bh[f][st], af[g][st], acc[f], 0, 0, 0);
            if constexpr (SPLIT) acc[f] = __builtin_amdgcn_mfma_f32_32x32x16_f16(bl[st], af[g][st], acc[f], 0, 0, 0);
          }
        const int64_t cb = czv + cbm[g];
        if constexpr (STG) {
          if (store_all) {
            uint32_t* sw = stg + (threadIdx.x >> 6) * 1024;
#pragma unroll
            for (int f = 0; f < NF; ++f)
#pragma unroll
              for (int v = 0; v < 16; v += 2) {
                const int nl = 16 * f + ((8 * (v >> 2) + 4 * (lane >> 5) + (v & 3)) >> 1);
                const int o = int(cbm[g] + cnT[nl]);
                unsigned bad;
                sw[o ^ (((o >> 6) & 15) << 2)] = CIO<_Float16>::pack(acc[f][v] * a.scale, acc[f][v + 1] * a.scale, bad);
                lsat += bad;
              }
            asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
            uint4* Cq = reinterpret_cast<uint4*>(reinterpret_cast<uint32_t*>(C) + czv);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int o = 4 * lane + 256 * r;
              Cq[lane + 64 * r] = *reinterpret_cast<const uint4*>(sw + (o ^ (((o >> 6) & 15) << 2)));
            }
            asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
            continue;
          }
        }
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
          for (int v = 0; v < 16; v += 2) {
            // rows 8 (v / 4) .. of the fragment: none of them is a result row
            // when 16 f + 4 (v / 4) >= N (the same in every lane)
            if (16 * f + 4 * (v >> 2) >= N) break;
            const int nl = 16 * f + ((8 * (v >> 2) + 4 * (lane >> 5) + (v & 3)) >> 1);
            const float re = acc[f][v] * a.scale, im = acc[f][v + 1] * a.scale;
            if (nl < N) {
              if (store_all) lsat += CIO<TO>::store(C, cb + cnT[nl], re, im);
              else lmax = fmaxf(lmax, fmaxf(fabsf(re), fabsf(im)));
            }
          }
      }
      if (nA != curA) {
        if constexpr (PIPE_A) {
#pragma unroll
          for (int g = 0; g < GPW; ++g)
#pragma unroll
            for (int st = 0; st < S; ++st) af[g][st] = an[g][st];
        } else {
          load_a(nA, af);
        }
      }
      curA = nA;
      curB = nB;
    }
  }
  block_amax_sat(lmax, lsat, a.amax, a.sat);
}

// waves: (2^nz / ZC) entry chunks x (M / 32 GPW) slabs; ZC = 16 consecutive
// entries per wave for batched steps with at least 2^8 entries, else one
// whether every entry's result is one contiguous block: the m and n strides
// are 1, 2, 4, ... in some order
static bool entry_block_contiguous(const GettArgs& a) {
  uint64_t seen = 0;
  const int nb = a.nm + a.nn;
  if (nb > 62) return false;
  for (int i = 0; i < nb; ++i) {
    const int64_t v = i < a.nm ? a.cm[i] : a.cn[i - a.nm];
    if (v <= 0 || (v & (v - 1)) || v >= (int64_t(1) << nb)) return false;
    seen |= uint64_t(v);
  }
  return seen == (uint64_t(1) << nb) - 1;
}

template <typename TB, typename TO, int KC, int GPW, int NF>
static hipError_t launch_skinny_g(const GettArgs& a, hipStream_t s) {
  if (((int64_t(1) << a.nm) % (32 * GPW)) != 0) return hipErrorInvalidValue;
  const int64_t slabs = (int64_t(1) << a.nm) / (32 * GPW);
  if (a.nz >= 8) {
    const int64_t n_waves = ((int64_t(1) << a.nz) / 16) * slabs;
    const int64_t blocks = (n_waves + 3) / 4;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    // B staged in LDS per chunk when every block's four waves share a chunk
    // and, for N <= 8, 16 / N entries through one B' fragment
    if constexpr (!std::is_same<TB, float>::value && NF == 1) {
      if (slabs % 4 == 0 && a.nn <= 3) {
        const dim3 g(static_cast<unsigned>(blocks)), b(256);
        if (a.nn == 0) hipLaunchKernelGGL((gett_skinny<TB, TO, KC, GPW, NF, 16, 8, 16>), g, b, 0, s, a, n_waves);
        else if (a.nn == 1) hipLaunchKernelGGL((gett_skinny<TB, TO, KC, GPW, NF, 16, 8, 8>), g, b, 0, s, a, n_waves);
        else if (a.nn == 2) hipLaunchKernelGGL((gett_skinny<TB, TO, KC, GPW, NF, 16, 8, 4>), g, b, 0, s, a, n_waves);
        else hipLaunchKernelGGL((gett_skinny<TB, TO, KC, GPW, NF, 16, 8, 2>), g, b, 0, s, a, n_waves);
        return hipGetLastError();
      }
    }
    if constexpr (GPW == 1 && NF == 2 && std::is_same<TO, _Float16>::value) {
      if (a.nm == 5 && a.nn == 5 && entry_block_contiguous(a)) {
        hipLaunchKernelGGL((gett_skinny<TB, TO, KC, 1, 2, 16, 0, 1, 1>), dim3(unsigned(blocks)), dim3(256), 0, s, a,
                           n_waves);
        return hipGetLastError();
      }
    }
    hipLaunchKernelGGL((gett_skinny<TB, TO, KC, GPW, NF, 16>), dim3(unsigned(blocks)), dim3(256), 0, s, a, n_waves);
  } else {
    const int64_t n_waves = (int64_t(1) << a.nz) * slabs;
    const int64_t blocks = (n_waves + 3) / 4;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((gett_skinny<TB, TO, KC, GPW, NF, 1>), dim3(unsigned(blocks)), dim3(256), 0, s, a, n_waves);
  }
  return hipGetLastError();
}

// GPW: 32-row groups per wave (fewer when M is smaller); NF = 2 for N > 16
template <typename TB, typename TO, int KC>
static hipError_t launch_skinny_k(const GettArgs& a, hipStream_t s) {
  constexpr int G = KC >= 64 ? 2 : 4;
  if (a.nn > 5 || a.nm < 5) return hipErrorInvalidValue;
  if (a.nn == 5) {
    if constexpr (std::is_same<TB, float>::value) {
      return hipErrorInvalidValue;
    } else {
      if constexpr (KC < 64) {
        if (a.nm >= 6) return launch_skinny_g<TB, TO, KC, 2, 2>(a, s);
      }
      return launch_skinny_g<TB, TO, KC, 1, 2>(a, s);
    }
  }
  if ((int64_t(1) << a.nm) >= 32 * G) return launch_skinny_g<TB, TO, KC, G, 1>(a, s);
  if (a.nm >= 6) return launch_skinny_g<TB, TO, KC, 2, 1>(a, s);
  return launch_skinny_g<TB, TO, KC, 1, 1>(a, s);
}

template <typename TB, typename TO>
static hipError_t launch_skinny(const GettArgs& a, hipStream_t s) {
  switch (a.nk) {
    case 2: return launch_skinny_k<TB, TO, 4>(a, s);
    case 3: return launch_skinny_k<TB, TO, 8>(a, s);
    case 4: return launch_skinny_k<TB, TO, 16>(a, s);
    case 5: return launch_skinny_k<TB, TO, 32>(a, s);
    case 6: return launch_skinny_k<TB, TO, 64>(a, s);
    default: return hipErrorInvalidValue;
  }
}

// ------------------------------------------------------------ launchers
// ------------------------------------------------------------ long-K MFMA
// Steps with a small result per batch entry (M, N <= 32 complex) and a long
// contraction (K >= 128 complex), e.g. the last stem steps that sum a
// 2^13-long index for each of 256 closed strings: one workgroup of 16 waves
// per batch entry.  Wave w takes the w-th contiguous sixteenth of K and runs
// MFMA 32x32x16 on fragments read straight from HBM (each lane 16 bytes of
// one A row and one B row per k step, four k steps in flight), B' formed in
// registers as in the DMA tile; the 16 partial 32 x 32 results are summed in
// LDS in wave order (fixed, so the result is deterministic).  HBM-bound: A
// and B are read once, the small C written once.
constexpr int LK_WAVES = 16;

template <typename TO>
__global__ void __launch_bounds__(64 * LK_WAVES) gett_longk(GettArgs a) {
  constexpr int U = 4;
  __shared__ float red[LK_WAVES][32][64];
  const int64_t M = int64_t(1) << a.nm, N = int64_t(1) << a.nn, K = int64_t(1) << a.nk;
  const int64_t z = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int r = lane & 31, half = lane >> 5;
  const bool okA = r < M, okB = r < N;
  const _Float16* A = static_cast<const _Float16*>(a.A);
  const _Float16* B = static_cast<const _Float16*>(a.B);
  // 16-byte chunks (4 complex) of row r; chunk 2t + half is this lane's part of k step t
  const uint4* pa = reinterpret_cast<const uint4*>(A + 2 * ((a.offA ? a.offA[z] : z * M * K) + (okA ? r : 0) * K));
  const uint4* pb = reinterpret_cast<const uint4*>(B + 2 * ((a.offB ? a.offB[z] : z * N * K) + (okB ? r : 0) * K));
  const int64_t steps = K / 8, per = steps / LK_WAVES;
  const int64_t t0 = int64_t(w) * per, t1 = t0 + per;
  f32x16 accr, acci;
#pragma unroll
  for (int v = 0; v < 16; ++v) { accr[v] = 0.0f; acci[v] = 0.0f; }
  auto step = [&](uint4 ra, uint4 rb) __attribute__((always_inline)) {
    u32x4 x, re, im;
    x[0] = rb.x; x[1] = rb.y; x[2] = rb.z; x[3] = rb.w;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      re[i] = x[i] ^ 0x80000000u;
      im[i] = __builtin_amdgcn_alignbit(x[i], x[i], 16);
    }
    const f16x8 av = __builtin_bit_cast(f16x8, ra);
    accr = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, re), av, accr, 0, 0, 0);
    acci = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, im), av, acci, 0, 0, 0);
  };
  // groups of U k steps, the loads of group g + 1 issued before the MFMAs of
  // group g (two register sets), so that two groups are in flight
  uint4 ra[2][U], rb[2][U];
  // rows past M (N) read row 0 and are zeroed by a mask: whole 16-byte
  // loads with no branch around them (a conditional load here became four
  // 4-byte loads, each behind its own branch)
  const uint32_t mA = okA ? ~0u : 0u, mB = okB ? ~0u : 0u;
  auto masked = [](uint4 x, uint32_t m) __attribute__((always_inline)) {
    x.x &= m;
    x.y &= m;
    x.z &= m;
    x.w &= m;
    return x;
  };
  auto load = [&](int set, int64_t t) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ra[set][u] = masked(pa[2 * (t + u) + half], mA);
      rb[set][u] = masked(pb[2 * (t + u) + half], mB);
    }
  };
  const int64_t groups = per / U;
  if (groups > 0) load(0, t0);
  for (int64_t g = 0; g < groups; g += 2) {
    if (g + 1 < groups) load(1, t0 + (g + 1) * U);
#pragma unroll
    for (int u = 0; u < U; ++u) step(ra[0][u], rb[0][u]);
    if (g + 1 < groups) {
      if (g + 2 < groups) load(0, t0 + (g + 2) * U);
#pragma unroll
      for (int u = 0; u < U; ++u) step(ra[1][u], rb[1][u]);
    }
  }
  for (int64_t t = t0 + groups * U; t < t1; ++t)
    step(masked(pa[2 * t + half], mA), masked(pb[2 * t + half], mB));
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    red[w][v][lane] = accr[v];
    red[w][16 + v][lane] = acci[v];
  }
  __syncthreads();
  // thread (v, l): the result of register v of lane l, summed over the waves
  const int v = tid >> 6, l = tid & 63;
  float re = 0.0f, im = 0.0f;
#pragma unroll
  for (int ww = 0; ww < LK_WAVES; ++ww) {
    re += red[ww][v][l];
    im += red[ww][16 + v][l];
  }
  re *= a.scale;
  im *= a.scale;
  const int m = l & 31, n = 8 * (v >> 2) + 4 * (l >> 5) + (v & 3);
  float lmax = 0.0f;
  unsigned lsat = 0;
  if (m < M && n < N) {
    lmax = fmaxf(fabsf(re), fabsf(im));
    if (!a.amax_only) {
      const int64_t off = scatter_bits(z, a.cz, a.nz) + scatter_bits(m, a.cm, a.nm) + scatter_bits(n, a.cn, a.nn);
      lsat = CIO<TO>::store(static_cast<TO*>(a.C), off, re, im);
    }
  }
  block_amax_sat(lmax, lsat, a.amax, a.sat);
}

template <typename TO>
static hipError_t launch_longk(const GettArgs& a, hipStream_t s) {
  const int64_t blocks = int64_t(1) << a.nz;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((gett_longk<TO>), dim3(unsigned(blocks)), dim3(64 * LK_WAVES), 0, s, a);
  return hipGetLastError();
}

bool kernel_applicable(int kernel, int in_dt, int nz, int nm, int nn, int nk) {
  (void)nz;
  (void)nk;
  if (kernel == K_THIN) return true;
  if (kernel == K_MFMA) return nm >= 5 && nn >= 4;
  if (kernel == K_MFMA_BIG || kernel == K_MFMA_BIG_X) return in_dt == 1 && nm >= 7 && nn >= 5;
  if (kernel == K_MFMA_DB_X || kernel == K_MFMA_WIDE_X) return in_dt == 1 && nm >= 7 && nn >= 6;
  if (kernel == K_MFMA_WIDE) return in_dt == 1 && nm >= 7 && nn >= 6;
  if (kernel == K_MFMA_DB || kernel == K_MFMA_DEEP) return in_dt == 1 && nm >= 7 && nn >= 6;
  if (kernel == K_NARROW) return nm >= 8 && nk <= 6 && nn <= 8 && nn + nk <= 8;
  if (kernel == K_SKINNY) return in_dt == 1 && nn <= 5 && nk >= 2 && nk <= 6 && nm >= 5;
  // whole 256 x 128 tiles, K a multiple of 32, and per-lane load offsets
  // (row * K * 4 bytes within a 256-row panel) that fit 32 bits
  if (kernel == K_MFMA_DMA || kernel == K_MFMA_DMA_X || kernel == K_MFMA_DMA4 || kernel == K_MFMA_DMA4_X)
    return in_dt == 1 && nm >= 8 && nn >= 7 && nk >= 5 && nk <= 21;
  if (kernel == K_MFMA_DMA2 || kernel == K_MFMA_DMA2_X) return in_dt == 1 && nm >= 7 && nn >= 7 && nk >= 5 && nk <= 21;
  // at least 8 complex per wave (one k step each)
  if (kernel == K_LONGK) return in_dt == 1 && nm <= 5 && nn <= 5 && nk >= 7;
  return false;
}

template <typename TA, typename TB, typename TO>
static hipError_t launch_thin(const GettArgs& a, hipStream_t s) {
  const int64_t blocks = thin_blocks(a);
  hipLaunchKernelGGL((gett_thin<TA, TB, TO>), dim3(unsigned(blocks)), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <typename TO, int WM, int WN, int MINB, int ST, int BK, int ORDER = 0>
static hipError_t launch_big(const GettArgs& a, hipStream_t s) {
  using T = BigTile<WM, WN>;
  const int64_t M = int64_t(1) << a.nm, N = int64_t(1) << a.nn, K = int64_t(1) << a.nk;
  const int64_t blocks = (int64_t(1) << a.nz) * ((M + T::BM - 1) / T::BM) * ((N + T::BN - 1) / T::BN);
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  const bool full = M % T::BM == 0 && N % T::BN == 0 && K % BK == 0;
  if (full)
    hipLaunchKernelGGL((gett_mfma_big<TO, WM, WN, MINB, ST, BK, true, ORDER>), dim3(unsigned(blocks)), dim3(256), 0, s,
                       a);
  else
    hipLaunchKernelGGL((gett_mfma_big<TO, WM, WN, MINB, ST, BK, false, ORDER>), dim3(unsigned(blocks)), dim3(256), 0,
                       s, a);
  return hipGetLastError();
}

template <typename TO, int ORDER, int NW, int BM = DMA_BM, int STAGES = 3>
static hipError_t launch_dma(const GettArgs& a, hipStream_t s) {
  if (a.nm < (BM == 256 ? 8 : 7) || a.nn < 7 || a.nk < 5 || a.nk > 21) return hipErrorInvalidValue;
  const int64_t blocks = (int64_t(1) << a.nz) * ((int64_t(1) << a.nm) / BM) * ((int64_t(1) << a.nn) / DMA_BN);
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((gett_mfma_dma<TO, ORDER, NW, BM, STAGES>), dim3(unsigned(blocks)), dim3(64 * NW), 0, s, a);
  return hipGetLastError();
}

template <typename TI, typename TO>
static hipError_t launch_typed(int kernel, const GettArgs& a, hipStream_t s) {
  if (kernel == K_THIN) return launch_thin<TI, TI, TO>(a, s);
  if (kernel == K_NARROW) return launch_narrow<TI, TI, TO>(a, s);
  if constexpr (std::is_same<TI, _Float16>::value) {
    if (kernel == K_SKINNY) return launch_skinny<_Float16, TO>(a, s);
    if (kernel == K_LONGK) return launch_longk<TO>(a, s);
  }
  const int64_t M = int64_t(1) << a.nm, N = int64_t(1) << a.nn;
  if (kernel == K_MFMA) {
    const int64_t blocks = (int64_t(1) << a.nz) * ((M + MF_BM - 1) / MF_BM) * ((N + MF_BN - 1) / MF_BN);
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((gett_mfma<TI, TO>), dim3(unsigned(blocks)), dim3(256), 0, s, a);
  } else {
    if constexpr (std::is_same<TI, _Float16>::value) {
      if (kernel == K_MFMA_DMA) return launch_dma<TO, 0, 8>(a, s);
      if (kernel == K_MFMA_DMA_X) return launch_dma<TO, 1, 8>(a, s);
      if (kernel == K_MFMA_DMA4) return launch_dma<TO, 0, 4>(a, s);
      if (kernel == K_MFMA_DMA4_X) return launch_dma<TO, 1, 4>(a, s);
      if (kernel == K_MFMA_DMA2) return launch_dma<TO, 0, 4, 128, 2>(a, s);
      if (kernel == K_MFMA_DMA2_X) return launch_dma<TO, 1, 4, 128, 2>(a, s);
      if (kernel == K_MFMA_BIG_X) return launch_big<TO, 4, 2, 2, 1, 32, 1>(a, s);
      if (kernel == K_MFMA_DB_X) return launch_big<TO, 4, 4, 1, 2, 32, 1>(a, s);
      if (kernel == K_MFMA_WIDE_X) return launch_big<TO, 4, 4, 1, 1, 32, 1>(a, s);
      if (kernel == K_MFMA_BIG) return launch_big<TO, 4, 2, 2, 1, 32>(a, s);
      if (kernel == K_MFMA_WIDE) return launch_big<TO, 4, 4, 1, 1, 32>(a, s);
      if (kernel == K_MFMA_DB) return launch_big<TO, 4, 4, 1, 2, 32>(a, s);
      return launch_big<TO, 4, 4, 1, 1, 64>(a, s);
    } else {
      return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

hipError_t launch_gett(int kernel, int a_dt, int b_dt, int out_dt, const GettArgs& a, hipStream_t s) {
  if (a_dt != b_dt) {
    // mixed operands: complex-half A with a complex64 B, streaming kernel only
    if (a_dt != 1 || b_dt != 0) return hipErrorInvalidValue;
    if (kernel == K_NARROW && kernel_applicable(K_NARROW, 1, a.nz, a.nm, a.nn, a.nk))
      return out_dt ? launch_narrow<_Float16, float, _Float16>(a, s) : launch_narrow<_Float16, float, float>(a, s);
    if (kernel == K_SKINNY && a.nn <= 4 && kernel_applicable(K_SKINNY, 1, a.nz, a.nm, a.nn, a.nk))
      return out_dt ? launch_skinny<float, _Float16>(a, s) : launch_skinny<float, float>(a, s);
    return out_dt ? launch_thin<_Float16, float, _Float16>(a, s) : launch_thin<_Float16, float, float>(a, s);
  }
  const int in_dt = a_dt;
  if (!kernel_applicable(kernel, in_dt, a.nz, a.nm, a.nn, a.nk)) kernel = K_THIN;
  if (in_dt == 0 && out_dt == 0) return launch_typed<float, float>(kernel, a, s);
  if (in_dt == 0 && out_dt == 1) return launch_typed<float, _Float16>(kernel, a, s);
  if (in_dt == 1 && out_dt == 0) return launch_typed<_Float16, float>(kernel, a, s);
  return launch_typed<_Float16, _Float16>(kernel, a, s);
}

// -------------------------------------------------------- slice copies
__global__ void __launch_bounds__(256) instantiate_kernel(const SliceCopy* tab, char* ws,
                                                          const int64_t* sigma_dev, int64_t sigma) {
  const SliceCopy e = tab[blockIdx.y];
  const int64_t sg = sigma_dev ? *sigma_dev : sigma;
  int64_t off = 0;
  for (int i = 0; i < e.nbits; ++i)
    if ((sg >> e.t[i]) & 1) off += e.stride[i];
  const char* src = ws + e.src + off;
  char* dst = ws + e.dst;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < e.n;
       i += int64_t(gridDim.x) * blockDim.x) {
    if (e.es == 8) reinterpret_cast<uint64_t*>(dst)[i] = reinterpret_cast<const uint64_t*>(src)[i];
    else reinterpret_cast<uint32_t*>(dst)[i] = reinterpret_cast<const uint32_t*>(src)[i];
  }
}

hipError_t launch_instantiate(const SliceCopy* tab, int n_entries, int64_t max_n, char* ws,
                              const int64_t* sigma_dev, int64_t sigma, hipStream_t s) {
  if (n_entries == 0) return hipSuccess;
  int64_t bx = (max_n + 255) / 256;
  if (bx > 1024) bx = 1024;
  if (bx < 1) bx = 1;
  hipLaunchKernelGGL(instantiate_kernel, dim3(unsigned(bx), unsigned(n_entries)), dim3(256), 0, s,
                     tab, ws, sigma_dev, sigma);
  return hipGetLastError();
}

// ---------------------------------------------------------- accumulate
// A slice is added only if no complex-half value of the plan saturated since
// the counter was last cleared: the steps of the slice ran before this
// kernel on the same stream, so a nonzero counter here means this slice (or
// an earlier one) was clamped.  The slice is then left out and the smallest
// such slice number is recorded, so the accumulator holds exactly the slices
// before the first saturated one.
// Each block takes chunks of 1024 values, a thread four of them 256 apart
// (every load and store instruction of a wave covers one contiguous piece:
// 256 B of the root, 1 KB of the accumulator as 16-byte complex128), with
// all four root loads issued before the read-modify-writes.
template <typename T>
__global__ void __launch_bounds__(256) accumulate_kernel(const T* root, double* out, int64_t n, int lbits,
                                                         const int64_t* rows, double scale,
                                                         const unsigned* sat, unsigned long long* first_bad,
                                                         const int64_t* sigma_dev, int64_t sigma) {
  if (sat && *sat) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      const int64_t sg = sigma_dev ? *sigma_dev : sigma;
      atomicMin(first_bad, (unsigned long long)sg);
    }
    return;
  }
  const int64_t mask = (int64_t(1) << lbits) - 1;
  double2* o = reinterpret_cast<double2*>(out);
  for (int64_t c = int64_t(blockIdx.x) * 1024; c < n; c += int64_t(gridDim.x) * 1024) {
    float re[4], im[4];
    int64_t d[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t i = c + v * 256 + threadIdx.x;
      d[v] = -1;
      re[v] = im[v] = 0.0f;
      if (i < n) {
        CIO<T>::load(root, i, re[v], im[v]);
        d[v] = rows ? (rows[i >> lbits] << lbits) | (i & mask) : i;
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v)
      if (d[v] >= 0) {
        double2 x = o[d[v]];
        x.x += double(re[v]) * scale;
        x.y += double(im[v]) * scale;
        o[d[v]] = x;
      }
  }
}

hipError_t launch_accumulate(int root_dt, const void* root, double* out, int64_t n, int lbits,
                             const int64_t* rows, double scale, const unsigned* sat,
                             unsigned long long* first_bad, const int64_t* sigma_dev, int64_t sigma,
                             hipStream_t s) {
  if (lbits < 0 || lbits > 62) return hipErrorInvalidValue;
  int64_t b = (n + 1023) / 1024;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  if (root_dt == 0)
    hipLaunchKernelGGL(accumulate_kernel<float>, dim3(unsigned(b)), dim3(256), 0, s,
                       static_cast<const float*>(root), out, n, lbits, rows, scale, sat, first_bad, sigma_dev,
                       sigma);
  else
    hipLaunchKernelGGL(accumulate_kernel<_Float16>, dim3(unsigned(b)), dim3(256), 0, s,
                       static_cast<const _Float16*>(root), out, n, lbits, rows, scale, sat, first_bad,
                       sigma_dev, sigma);
  return hipGetLastError();
}

__global__ void set_i64_kernel(int64_t* p, int64_t v) { *p = v; }
__global__ void add_i64_kernel(int64_t* p, int64_t v) { *p += v; }
__global__ void zero_u32_kernel(unsigned* p, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    p[i] = 0u;
}

hipError_t launch_set_i64(int64_t* p, int64_t v, hipStream_t s) {
  hipLaunchKernelGGL(set_i64_kernel, dim3(1), dim3(1), 0, s, p, v);
  return hipGetLastError();
}
hipError_t launch_add_i64(int64_t* p, int64_t v, hipStream_t s) {
  hipLaunchKernelGGL(add_i64_kernel, dim3(1), dim3(1), 0, s, p, v);
  return hipGetLastError();
}
hipError_t launch_zero_u32(unsigned* p, int64_t n, hipStream_t s) {
  int64_t b = (n + 255) / 256;
  if (b > 1024) b = 1024;
  if (b < 1) b = 1;
  hipLaunchKernelGGL(zero_u32_kernel, dim3(unsigned(b)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------- top-k
// One workgroup per group.  Round r finds the best entry strictly after the
// (r-1)-th selection in the order (p descending, position ascending):
// per-lane scan, wave shuffle reduction, then across the four waves.
__device__ __forceinline__ bool topk_better(double p, int64_t j, double q, int64_t i) {
  return p > q || (p == q && j < i);
}

__global__ void __launch_bounds__(256) topk_kernel(const double* amps, int64_t group_size, int k,
                                                   int64_t* out_idx, double* out_prob) {
  __shared__ double sp[4];
  __shared__ int64_t sj[4];
  const int64_t g = blockIdx.x;
  const double* base = amps + 2 * g * group_size;
  double prev_p = 0.0;
  int64_t prev_j = -1;
  bool have_prev = false;
  for (int r = 0; r < k; ++r) {
    double bp = -1.0;
    int64_t bj = INT64_MAX;
    for (int64_t j = threadIdx.x; j < group_size; j += blockDim.x) {
      const double re = base[2 * j], im = base[2 * j + 1];
      const double p = prob_of(re, im);
      const bool after = !have_prev || p < prev_p || (p == prev_p && j > prev_j);
      if (after && topk_better(p, j, bp, bj)) { bp = p; bj = j; }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double op = __shfl_xor(bp, o);
      const int64_t oj = __shfl_xor(bj, o);
      if (topk_better(op, oj, bp, bj)) { bp = op; bj = oj; }
    }
    if ((threadIdx.x & 63) == 0) { sp[threadIdx.x >> 6] = bp; sj[threadIdx.x >> 6] = bj; }
    __syncthreads();
    double fp = sp[0];
    int64_t fj = sj[0];
    for (int i = 1; i < int(blockDim.x >> 6); ++i)
      if (topk_better(sp[i], sj[i], fp, fj)) { fp = sp[i]; fj = sj[i]; }
    __syncthreads();
    if (threadIdx.x == 0) {
      out_idx[g * k + r] = fj;
      out_prob[g * k + r] = fp;
    }
    prev_p = fp;
    prev_j = fj;
    have_prev = true;
  }
}

hipError_t launch_topk(const double* amps, int64_t n_groups, int64_t group_size, int k,
                       int64_t* out_idx, double* out_prob, hipStream_t s) {
  if (n_groups <= 0) return hipSuccess;
  if (n_groups > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(topk_kernel, dim3(unsigned(n_groups)), dim3(256), 0, s, amps, group_size, k,
                     out_idx, out_prob);
  return hipGetLastError();
}

}  // namespace lf
