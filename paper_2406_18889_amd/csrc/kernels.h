// Device kernels of the contraction path (gfx950).  Launch wrappers only;
// see kernels.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lf {

constexpr int MAXZ = 24;
constexpr int MAXMN = 40;

// One pairwise contraction C[z,m,n] = sum_k A[z,m,k] * B[z,n,k] over complex
// numbers stored as (re, im) pairs.  A is read as a row-major
// [2^nz][2^nm][2^nk] array, B as [2^nz][2^nn][2^nk]; C element (z,m,n) is at
// sum of the strides of the set bits of z, m and n (cz, cm, cn; bit 0 the
// least significant), so the result lands in any index order without a
// permutation pass.  The accumulated value is multiplied by `scale`
// (a power of two) before it is stored.
//
// In a batched product the [m][k] block of A for batch entry z starts at
// element offA[z] (and B's [n][k] block at offB[z]); a null table means the
// plain row-major position z * 2^(nm+nk) (z * 2^(nn+nk)).
struct GettArgs {
  const void* A;
  const void* B;
  void* C;
  const int64_t* offA;
  const int64_t* offB;
  int nz, nm, nn, nk;
  float scale;
  int amax_only;      // 1: record the largest |re|,|im| only, store nothing
  float* amax;        // nullable: running max of |re|,|im| of stored values (as bits)
  unsigned* sat;      // nullable: count of values clamped to the half range
  int64_t cz[MAXZ];
  int64_t cm[MAXMN];
  int64_t cn[MAXMN];
};

// K_THIN: streaming, one row per thread, any shape; K_MFMA: 128 x 64 complex
// tile (both arithmetics); K_MFMA_BIG: 256 x 64 complex tile, complex-half
// only; K_NARROW: one row per thread with B staged in LDS, for N K <= 256
// and M >= 256; K_MFMA_WIDE: 256 x 128 complex tile, complex-half only;
// K_MFMA_DB: the 256 x 128 tile with double-buffered LDS, complex-half
// only; K_MFMA_DEEP: the 256 x 128 tile with 64-deep K steps (one LDS
// buffer).
// K_SKINNY: MFMA on 32-row groups of A against a B' of at most 32 rows held
// in registers (N <= 16, 4 <= K <= 64), complex-half A, B either type.
// K_MFMA_BIG_X, K_MFMA_DB_X, K_MFMA_WIDE_X: kernels 2, 5 and 4 with the XCD-grouped tile order
// K_MFMA_DMA: the 256 x 128 tile with eight waves and operands loaded straight
// into a three-stage LDS ring, whole tiles only, complex-half only;
// K_MFMA_DMA_X: the same with the XCD-grouped tile order; K_MFMA_DMA4,
// K_MFMA_DMA4_X: kernels 11 and 12 on four waves (one per SIMD, 128 m x 64 n each)
// (each XCD a contiguous range of tiles, groups of 8 m-tiles sweeping n):
// less HBM traffic when an A panel would otherwise be fetched by every XCD.
// K_LONGK: M, N <= 32 complex and K >= 128: one 16-wave workgroup per batch
// entry, K split over the waves, complex-half only.
// K_MFMA_DMA2, K_MFMA_DMA2_X: the 128 x 128 tile of the DMA-fed kernel on
// four waves with two operand stages (two workgroups per CU), both tile
// orders; whole tiles (M % 128, N % 128, K % 32 == 0).
enum KernelId : int {
  K_THIN = 0, K_MFMA = 1, K_MFMA_BIG = 2, K_NARROW = 3, K_MFMA_WIDE = 4, K_MFMA_DB = 5, K_MFMA_DEEP = 6,
  K_SKINNY = 7, K_MFMA_BIG_X = 8, K_MFMA_DB_X = 9, K_MFMA_WIDE_X = 10, K_MFMA_DMA = 11,
  K_MFMA_DMA_X = 12, K_MFMA_DMA4 = 13, K_MFMA_DMA4_X = 14, K_LONGK = 15, K_MFMA_DMA2 = 16,
  K_MFMA_DMA2_X = 17, K_COUNT = 18
};

// a_dt, b_dt, out_dt: 0 complex64 (float pairs), 1 complex-half (_Float16
// pairs).  a_dt != b_dt is allowed only as a complex-half A with a
// complex64 B, on the streaming kernels and K_SKINNY.
hipError_t launch_gett(int kernel, int a_dt, int b_dt, int out_dt, const GettArgs& a, hipStream_t s);

// One step of a grouped launch of small streaming steps (the streaming
// one-row-per-thread kernel): its arguments, its operand and result types
// (combo = a_dt | b_dt << 1 | out_dt << 2, 1 = complex-half; B complex-half
// only with A complex-half) and its block count.
struct GroupStep {
  GettArgs a;
  int32_t combo;
  int32_t pad;
  int64_t blocks;
};
// blocks of the streaming kernel's launch for these arguments
int64_t thin_blocks(const GettArgs& a);
// the n steps of tab (device memory) in one launch of total_blocks blocks
// (the sum of their block counts)
hipError_t launch_thin_group(const GroupStep* tab, int n, int64_t total_blocks, hipStream_t s);
bool kernel_applicable(int kernel, int in_dt, int nz, int nm, int nn, int nk);

// Copies of the slice-dependent blocks of leaf tensors.
struct SliceCopy {
  int64_t src;        // byte offset in the workspace of the full leaf
  int64_t dst;        // byte offset of the per-slice copy
  int64_t n;          // elements per slice block
  int32_t es;         // element bytes (8 complex64, 4 complex-half)
  int32_t nbits;      // sliced wires in this leaf
  int32_t t[8];       // slice-number bit of each
  int64_t stride[8];  // byte stride of each in the full leaf
};
hipError_t launch_instantiate(const SliceCopy* tab, int n_entries, int64_t max_n, char* ws,
                              const int64_t* sigma_dev, int64_t sigma, hipStream_t s);

// out[d(i)] += root[i] * scale for i < n (complex128 accumulator, float64
// math), where root rows hold 2^lbits values and d maps row z to row
// rows[z] (d(i) = i when rows is null), unless *sat is nonzero (a
// complex-half value of this slice or an earlier one saturated): then
// nothing is added and *first_bad = min(*first_bad, slice number), the slice
// number read from *sigma_dev when it is not null.
hipError_t launch_accumulate(int root_dt, const void* root, double* out, int64_t n, int lbits,
                             const int64_t* rows, double scale, const unsigned* sat,
                             unsigned long long* first_bad, const int64_t* sigma_dev, int64_t sigma,
                             hipStream_t s);

hipError_t launch_set_i64(int64_t* p, int64_t v, hipStream_t s);
hipError_t launch_add_i64(int64_t* p, int64_t v, hipStream_t s);
hipError_t launch_zero_u32(unsigned* p, int64_t n, hipStream_t s);

// p = re*re + im*im with each product and the sum rounded separately (the
// compiler must not fuse them into a multiply-add)
__device__ __forceinline__ double prob_of(double re, double im) {
#pragma clang fp contract(off)
  const double rr = re * re;
  const double ii = im * im;
  return rr + ii;
}

// select.hip: selection at any size (radix select, ordered compaction,
// stable sort); scratch of select_scratch_bytes(k) bytes, 256-byte aligned
uint64_t select_scratch_bytes(int64_t k);
bool select_uses_radix(int64_t group_size, int k);
hipError_t launch_select(const double* amps, int64_t n_groups, int64_t group_size, int64_t k,
                         int64_t* out_idx, double* out_prob, void* scratch, hipStream_t s);

hipError_t launch_topk(const double* amps, int64_t n_groups, int64_t group_size, int k,
                       int64_t* out_idx, double* out_prob, hipStream_t s);

}  // namespace lf
