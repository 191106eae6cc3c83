// Top-k post-selection at any size (Methods A: the k strings of S~ with the
// largest p, over all of S~ or per group of correlated strings).
//
// Order: p descending, then position ascending, with p = fl(fl(re*re) +
// fl(im*im)) in float64.  Because p >= 0, the bit pattern of p read as an
// unsigned 64-bit integer orders exactly as p does, so the selection works on
// those keys:
//
//  1. radix selection of the k-th largest key, twelve bits at a time from
//     the top (five levels of 12 bits and one of 4): each level histograms
//     the keys that share the bits fixed so far (one pass over the
//     amplitudes), and a single-workgroup pass picks the digit holding the
//     k-th element.  Everything above that digit is taken; the search stops
//     as soon as the elements of the chosen digit are exactly the ones still
//     needed, else continues inside the digit.  After the last level the
//     remaining class is one exact key (ties): the lowest positions win.
//  2. ordered compaction: one pass counts, per contiguous chunk, the keys
//     above the class and the keys in it; an exclusive scan over the chunks
//     gives each chunk its output offset, and a second pass writes the
//     selected (key, position) pairs in position order.
//  3. stable least-significant-digit radix sort of the k pairs by key,
//     descending, four bits per pass (sixteen passes): equal keys keep their
//     position order.
//
// All of it runs on the device with no host synchronisation in between; the
// state of the selection lives in device memory (scratch).  Memory traffic:
// up to six histogram passes plus two compaction passes over the 16-byte
// amplitudes (most inputs stop after two or three levels), then 16 passes
// over 16 k bytes.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/leapfrog.h"
#include "kernels.h"

namespace lf {

lf_status set_error(lf_status s, const std::string& msg);  // runtime.hip

namespace {

struct SelState {
  unsigned long long prefix;       // key bits fixed so far
  unsigned long long mask;         // which bits those are
  unsigned long long need;         // elements still to take from the class
  unsigned long long above;        // elements above the class (all taken)
  unsigned long long class_count;  // elements whose fixed bits equal prefix
  int level;
  int done;
};

constexpr int SEL_LEVELS = 6;
constexpr int SEL_BINS = 4096;
constexpr int SEL_CHUNKS = 4096;  // compaction chunks (upper bound)
constexpr int SORT_TILE = 1024;   // items per sort block (256 threads x 4)

__host__ __device__ constexpr int sel_shift(int level) { return level < 5 ? 52 - 12 * level : 0; }
__host__ __device__ constexpr int sel_width(int level) { return level < 5 ? 12 : 4; }

__device__ __forceinline__ unsigned long long key_at(const double* amps, int64_t i) {
  const double2 v = reinterpret_cast<const double2*>(amps)[i];
  return static_cast<unsigned long long>(__double_as_longlong(prob_of(v.x, v.y)));
}

__device__ __forceinline__ unsigned long long lanes_below() {
  return (1ull << (threadIdx.x & 63)) - 1ull;
}

__global__ void sel_init_kernel(SelState* st, unsigned long long* hist, unsigned long long k,
                                unsigned long long n) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->prefix = 0;
    st->mask = 0;
    st->need = k;
    st->above = 0;
    st->class_count = n;
    st->level = 0;
    st->done = k == n ? 1 : 0;
  }
  for (int i = threadIdx.x; i < SEL_BINS; i += blockDim.x) hist[i] = 0;
}

// histogram of the next digit over the keys that match the fixed bits
__global__ void __launch_bounds__(256) sel_hist_kernel(const double* amps, int64_t n,
                                                       const SelState* st,
                                                       unsigned long long* hist) {
  if (st->done) return;
  __shared__ unsigned h[SEL_BINS];
  for (int i = threadIdx.x; i < SEL_BINS; i += 256) h[i] = 0;
  __syncthreads();
  const unsigned long long pre = st->prefix, msk = st->mask;
  const int L = st->level;
  const int sh = sel_shift(L);
  const unsigned dm = (1u << sel_width(L)) - 1u;
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const unsigned long long k = key_at(amps, i);
    if ((k & msk) == pre) atomicAdd(&h[unsigned(k >> sh) & dm], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < SEL_BINS; i += 256)
    if (h[i]) atomicAdd(&hist[i], static_cast<unsigned long long>(h[i]));
}

// one workgroup: the digit that holds the need-th largest remaining key
__global__ void __launch_bounds__(256) sel_pick_kernel(SelState* st, unsigned long long* hist) {
  if (st->done) return;
  __shared__ unsigned long long tsum[256];
  const int L = st->level;
  const unsigned long long need = st->need;  // read before any thread writes the state
  const int nb = 1 << sel_width(L);
  const int per = nb >= 256 ? nb / 256 : 1;
  const int t = threadIdx.x;
  // thread t owns digits [nb - per (t + 1), nb - per t), highest first
  unsigned long long s = 0;
  const int top = nb - per * t;
  for (int d = top - 1; d >= top - per && d >= 0; --d) s += hist[d];
  tsum[t] = s;
  __syncthreads();
  // inclusive scan over threads (descending digit order)
  for (int o = 1; o < 256; o <<= 1) {
    const unsigned long long v = t >= o ? tsum[t - o] : 0ull;
    __syncthreads();
    tsum[t] += v;
    __syncthreads();
  }
  const unsigned long long before = tsum[t] - s;  // keys in higher digits
  if (top > 0 && before < need && need <= tsum[t]) {
    unsigned long long run = before;
    for (int d = top - 1; d >= top - per && d >= 0; --d) {
      const unsigned long long h = hist[d];
      if (run + h >= need) {
        const int sh = sel_shift(L);
        st->above += run;
        st->need = need - run;
        st->prefix |= static_cast<unsigned long long>(d) << sh;
        st->mask |= static_cast<unsigned long long>(nb - 1) << sh;
        st->class_count = h;
        st->level = L + 1;
        st->done = (h == need - run || L + 1 == SEL_LEVELS) ? 1 : 0;
        break;
      }
      run += h;
    }
  }
  __syncthreads();
  for (int i = t; i < SEL_BINS; i += 256) hist[i] = 0;
}

__device__ __forceinline__ unsigned long long block_sum(unsigned long long v, unsigned long long* sm) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = v;
  __syncthreads();
  v = sm[0] + sm[1] + sm[2] + sm[3];
  __syncthreads();
  return v;
}

// per chunk: keys above the class, keys in the class
__global__ void __launch_bounds__(256) sel_count_kernel(const double* amps, int64_t n, int64_t chunk,
                                                        const SelState* st,
                                                        unsigned long long* cnt) {
  __shared__ unsigned long long sm[4];
  const int64_t b0 = int64_t(blockIdx.x) * chunk;
  const int64_t b1 = b0 + chunk < n ? b0 + chunk : n;
  const unsigned long long pre = st->prefix, msk = st->mask, hi = pre | ~msk;
  unsigned long long sure = 0, cls = 0;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += 256) {
    const unsigned long long k = key_at(amps, i);
    sure += k > hi ? 1 : 0;
    cls += (k & msk) == pre ? 1 : 0;
  }
  sure = block_sum(sure, sm);
  cls = block_sum(cls, sm);
  if (threadIdx.x == 0) {
    cnt[2 * blockIdx.x] = sure;
    cnt[2 * blockIdx.x + 1] = cls;
  }
}

// one workgroup: exclusive scan of the chunk counts (pairs), in place
__global__ void __launch_bounds__(256) sel_scan_kernel(unsigned long long* cnt, int nchunks) {
  __shared__ unsigned long long ts[2][256];
  const int t = threadIdx.x;
  const int per = (nchunks + 255) / 256;
  const int c0 = t * per;
  const int c1 = c0 + per < nchunks ? c0 + per : nchunks;
  unsigned long long a = 0, b = 0;
  for (int c = c0; c < c1; ++c) {
    a += cnt[2 * c];
    b += cnt[2 * c + 1];
  }
  ts[0][t] = a;
  ts[1][t] = b;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    const unsigned long long va = t >= o ? ts[0][t - o] : 0ull;
    const unsigned long long vb = t >= o ? ts[1][t - o] : 0ull;
    __syncthreads();
    ts[0][t] += va;
    ts[1][t] += vb;
    __syncthreads();
  }
  unsigned long long ra = ts[0][t] - a, rb = ts[1][t] - b;
  for (int c = c0; c < c1; ++c) {
    const unsigned long long x = cnt[2 * c], y = cnt[2 * c + 1];
    cnt[2 * c] = ra;
    cnt[2 * c + 1] = rb;
    ra += x;
    rb += y;
  }
}

// writes the selected (p, position) pairs of each chunk in position order
__global__ void __launch_bounds__(256) sel_compact_kernel(const double* amps, int64_t n, int64_t chunk,
                                                          const SelState* st,
                                                          const unsigned long long* off,
                                                          double* out_p, int64_t* out_j, int64_t k_out) {
  __shared__ unsigned wsel[4], wcls[4];
  const int64_t b0 = int64_t(blockIdx.x) * chunk;
  const int64_t b1 = b0 + chunk < n ? b0 + chunk : n;
  const unsigned long long pre = st->prefix, msk = st->mask, hi = pre | ~msk, need = st->need;
  unsigned long long cls_run = off[2 * blockIdx.x + 1];
  unsigned long long sel_run = off[2 * blockIdx.x] + (cls_run < need ? cls_run : need);
  const int w = threadIdx.x >> 6;
  for (int64_t base = b0; base < b1; base += 256) {
    const int64_t i = base + threadIdx.x;
    const bool in = i < b1;
    const unsigned long long k = in ? key_at(amps, i) : 0ull;
    const bool c = in && (k & msk) == pre;
    const unsigned long long bc = __ballot(c);
    if ((threadIdx.x & 63) == 0) wcls[w] = __popcll(bc);
    __syncthreads();
    unsigned cls_before = 0;
    for (int v = 0; v < w; ++v) cls_before += wcls[v];
    const unsigned long long rank = cls_run + cls_before + __popcll(bc & lanes_below());
    const bool take = in && (k > hi || (c && rank < need));
    const unsigned long long bt = __ballot(take);
    if ((threadIdx.x & 63) == 0) wsel[w] = __popcll(bt);
    __syncthreads();
    unsigned sel_before = 0;
    for (int v = 0; v < w; ++v) sel_before += wsel[v];
    const unsigned long long pos = sel_run + sel_before + __popcll(bt & lanes_below());
    if (take && pos < static_cast<unsigned long long>(k_out)) {  // exactly k are taken
      out_p[pos] = __longlong_as_double(static_cast<long long>(k));
      out_j[pos] = i;
    }
    sel_run += wsel[0] + wsel[1] + wsel[2] + wsel[3];
    cls_run += wcls[0] + wcls[1] + wcls[2] + wcls[3];
    __syncthreads();
  }
}

__device__ __forceinline__ int desc_digit(double p, int shift) {
  const unsigned long long k = static_cast<unsigned long long>(__double_as_longlong(p));
  return 15 - int((k >> shift) & 15ull);
}

// per sort tile: counts of each (descending) digit, digit-major [16][ntiles]
__global__ void __launch_bounds__(256) sort_count_kernel(const double* keys, int64_t m, int shift,
                                                         unsigned* cnt, int ntiles) {
  __shared__ unsigned c[16];
  if (threadIdx.x < 16) c[threadIdx.x] = 0;
  __syncthreads();
  for (int s = 0; s < SORT_TILE / 256; ++s) {
    const int64_t i = int64_t(blockIdx.x) * SORT_TILE + s * 256 + threadIdx.x;
    if (i < m) atomicAdd(&c[desc_digit(keys[i], shift)], 1u);
  }
  __syncthreads();
  if (threadIdx.x < 16) cnt[threadIdx.x * ntiles + blockIdx.x] = c[threadIdx.x];
}

// one workgroup: exclusive scan of n counts, in place
__global__ void __launch_bounds__(256) sort_scan_kernel(unsigned* cnt, int n) {
  __shared__ unsigned ts[256];
  const int t = threadIdx.x;
  const int per = (n + 255) / 256;
  const int c0 = t * per;
  const int c1 = c0 + per < n ? c0 + per : n;
  unsigned a = 0;
  for (int c = c0; c < c1; ++c) a += cnt[c];
  ts[t] = a;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    const unsigned v = t >= o ? ts[t - o] : 0u;
    __syncthreads();
    ts[t] += v;
    __syncthreads();
  }
  unsigned r = ts[t] - a;
  for (int c = c0; c < c1; ++c) {
    const unsigned x = cnt[c];
    cnt[c] = r;
    r += x;
  }
}

// stable scatter: items of a tile in order (sub-tile, wave, lane)
__global__ void __launch_bounds__(256) sort_scatter_kernel(const double* kin, const int64_t* jin,
                                                           double* kout, int64_t* jout, int64_t m,
                                                           int shift, const unsigned* off, int ntiles) {
  __shared__ unsigned base[16];
  __shared__ unsigned wc[4][16];
  const int w = threadIdx.x >> 6;
  if (threadIdx.x < 16) base[threadIdx.x] = off[threadIdx.x * ntiles + blockIdx.x];
  __syncthreads();
  for (int s = 0; s < SORT_TILE / 256; ++s) {
    const int64_t i = int64_t(blockIdx.x) * SORT_TILE + s * 256 + threadIdx.x;
    const bool in = i < m;
    const double kv = in ? kin[i] : 0.0;
    const int64_t jv = in ? jin[i] : 0;
    const int d = in ? desc_digit(kv, shift) : -1;
    unsigned long long mine = 0;
    for (int v = 0; v < 16; ++v) {
      const unsigned long long bv = __ballot(d == v);
      if ((threadIdx.x & 63) == 0) wc[w][v] = __popcll(bv);
      if (d == v) mine = bv;
    }
    __syncthreads();
    if (in) {
      unsigned pos = base[d] + __popcll(mine & lanes_below());
      for (int v = 0; v < w; ++v) pos += wc[v][d];
      if (pos < m) {  // the counts place every item inside [0, m)
        kout[pos] = kv;
        jout[pos] = jv;
      }
    }
    __syncthreads();
    if (threadIdx.x < 16) base[threadIdx.x] += wc[0][threadIdx.x] + wc[1][threadIdx.x] +
                                               wc[2][threadIdx.x] + wc[3][threadIdx.x];
    __syncthreads();
  }
}

// q[r] = p of element idx[r] (NaN for an index outside [0, n))
__global__ void __launch_bounds__(256) probs_at_kernel(const double* amps, int64_t n, const int64_t* idx,
                                                       int64_t m, double* out) {
  const int64_t r = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (r >= m) return;
  const int64_t i = idx[r];
  if (i < 0 || i >= n) {
    out[r] = __longlong_as_double(0x7ff8000000000000ll);
    return;
  }
  const double re = amps[2 * i], im = amps[2 * i + 1];
  out[r] = prob_of(re, im);
}

}  // namespace

uint64_t select_scratch_bytes(int64_t k) {
  const int64_t ntiles = (k + SORT_TILE - 1) / SORT_TILE;
  return 256 + 8ull * SEL_BINS + 16ull * SEL_CHUNKS + 4ull * 16 * uint64_t(ntiles) + 16ull * uint64_t(k) + 256;
}

bool select_uses_radix(int64_t group_size, int k) { return group_size > 65536 || k > 1024; }

// Selection of every group with the radix path, scratch of at least
// select_scratch_bytes(k) bytes at `scratch` (256-byte aligned).
hipError_t launch_select(const double* amps, int64_t n_groups, int64_t group_size, int64_t k,
                         int64_t* out_idx, double* out_prob, void* scratch, hipStream_t s) {
  char* p = static_cast<char*>(scratch);
  SelState* st = reinterpret_cast<SelState*>(p);
  unsigned long long* hist = reinterpret_cast<unsigned long long*>(p + 256);
  unsigned long long* cnt = hist + SEL_BINS;
  const int64_t ntiles = (k + SORT_TILE - 1) / SORT_TILE;
  unsigned* scnt = reinterpret_cast<unsigned*>(cnt + 2 * SEL_CHUNKS);
  char* q = reinterpret_cast<char*>(scnt + 16 * ntiles);
  q += (256 - reinterpret_cast<uintptr_t>(q) % 256) % 256;
  double* tkey = reinterpret_cast<double*>(q);
  int64_t* tidx = reinterpret_cast<int64_t*>(q + 8 * k);
  const int64_t n = group_size;
  int64_t nchunks = (n + 1023) / 1024;
  if (nchunks > SEL_CHUNKS) nchunks = SEL_CHUNKS;
  int64_t chunk = (n + nchunks - 1) / nchunks;
  chunk = (chunk + 255) / 256 * 256;
  nchunks = (n + chunk - 1) / chunk;
  int64_t hblocks = (n + 255) / 256;
  if (hblocks > 4096) hblocks = 4096;
  for (int64_t g = 0; g < n_groups; ++g) {
    const double* a = amps + 2 * g * group_size;
    double* op = out_prob + g * k;
    int64_t* oj = out_idx + g * k;
    hipLaunchKernelGGL(sel_init_kernel, dim3(1), dim3(256), 0, s, st, hist,
                       static_cast<unsigned long long>(k), static_cast<unsigned long long>(n));
    for (int L = 0; L < SEL_LEVELS; ++L) {
      hipLaunchKernelGGL(sel_hist_kernel, dim3(unsigned(hblocks)), dim3(256), 0, s, a, n, st, hist);
      hipLaunchKernelGGL(sel_pick_kernel, dim3(1), dim3(256), 0, s, st, hist);
    }
    hipLaunchKernelGGL(sel_count_kernel, dim3(unsigned(nchunks)), dim3(256), 0, s, a, n, chunk, st, cnt);
    hipLaunchKernelGGL(sel_scan_kernel, dim3(1), dim3(256), 0, s, cnt, int(nchunks));
    hipLaunchKernelGGL(sel_compact_kernel, dim3(unsigned(nchunks)), dim3(256), 0, s, a, n, chunk, st, cnt,
                       op, oj, k);
    // sixteen stable passes, out -> tmp -> out ...; the result ends in out
    for (int pass = 0; pass < 16; ++pass) {
      const double* kin = (pass & 1) ? tkey : op;
      const int64_t* jin = (pass & 1) ? tidx : oj;
      double* kout = (pass & 1) ? op : tkey;
      int64_t* jout = (pass & 1) ? oj : tidx;
      hipLaunchKernelGGL(sort_count_kernel, dim3(unsigned(ntiles)), dim3(256), 0, s, kin, k, 4 * pass,
                         scnt, int(ntiles));
      hipLaunchKernelGGL(sort_scan_kernel, dim3(1), dim3(256), 0, s, scnt, int(16 * ntiles));
      hipLaunchKernelGGL(sort_scatter_kernel, dim3(unsigned(ntiles)), dim3(256), 0, s, kin, jin, kout, jout,
                         k, 4 * pass, scnt, int(ntiles));
    }
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- fixed scratch
constexpr uint64_t NOALLOC_SCRATCH_BYTES = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

int64_t noalloc_max_k() {
  int64_t k = int64_t(NOALLOC_SCRATCH_BYTES / 17);
  while (k > 1 && select_scratch_bytes(k) > NOALLOC_SCRATCH_BYTES) --k;
  return k;
}

// device address of `scratch` on the current device, looked up once per device
lf_status noalloc_scratch(void** out) {
  static std::mutex mu;
  static std::vector<void*> ptr;  // indexed by device
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return set_error(LF_HIP_ERROR, std::string("hipGetDevice: ") + hipGetErrorString(e));
  std::lock_guard<std::mutex> lk(mu);
  if (dev >= int(ptr.size())) ptr.resize(dev + 1, nullptr);
  if (!ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_error(LF_HIP_ERROR, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    ptr[dev] = p;
  }
  *out = ptr[dev];
  return LF_OK;
}

}  // namespace lf

using lf::set_error;

extern "C" {

lf_status lf_postselect_topk(const void* amps, int64_t n_groups, int64_t group_size, int32_t k,
                             int64_t* out_idx, double* out_prob, void* stream) {
  if (n_groups < 0) return set_error(LF_INVALID_ARGUMENT, "n_groups < 0");
  if (n_groups == 0) return LF_OK;
  if (!amps || !out_idx || !out_prob) return set_error(LF_INVALID_ARGUMENT, "NULL pointer");
  if (reinterpret_cast<uintptr_t>(amps) % 16 != 0)
    return set_error(LF_INVALID_ARGUMENT, "amps must be 16-byte aligned");
  if (group_size < 1 || group_size > (int64_t(1) << 40))
    return set_error(LF_INVALID_ARGUMENT, "group_size out of range");
  if (n_groups > (int64_t(1) << 40) / group_size)
    return set_error(LF_INVALID_ARGUMENT, "n_groups * group_size above 2^40");
  if (k < 1 || k > group_size) return set_error(LF_INVALID_ARGUMENT, "k out of range");
  if (int64_t(k) * n_groups > (int64_t(1) << 31))
    return set_error(LF_INVALID_ARGUMENT, "n_groups * k above 2^31");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const double* a = static_cast<const double*>(amps);
  if (!lf::select_uses_radix(group_size, k)) {
    hipError_t e = lf::launch_topk(a, n_groups, group_size, k, out_idx, out_prob, st);
    if (e != hipSuccess) return set_error(LF_HIP_ERROR, std::string("top-k launch: ") + hipGetErrorString(e));
    return LF_OK;
  }
  void* scratch = nullptr;
  hipError_t e = hipMalloc(&scratch, lf::select_scratch_bytes(k));
  if (e != hipSuccess) return set_error(LF_HIP_ERROR, std::string("top-k scratch: ") + hipGetErrorString(e));
  e = lf::launch_select(a, n_groups, group_size, k, out_idx, out_prob, scratch, st);
  hipError_t e2 = hipStreamSynchronize(st);
  (void)hipFree(scratch);
  if (e == hipSuccess) e = e2;
  if (e != hipSuccess) return set_error(LF_HIP_ERROR, std::string("top-k selection: ") + hipGetErrorString(e));
  return LF_OK;
}

// Entry point for callers that cannot allocate (stream capture, serving
// loops): the radix path's scratch is a file-scope device array of fixed
// size, one copy per GPU, addressed through the pointer that
// hipGetSymbolAddress returns on that device (the array's name in host code
// is not a device address).
lf_status lf_postselect_topk_noalloc(const void* amps, int64_t n_groups, int64_t group_size, int32_t k,
                                     int64_t* out_idx, double* out_prob, void* stream) {
  if (n_groups < 0) return set_error(LF_INVALID_ARGUMENT, "n_groups < 0");
  if (n_groups == 0) return LF_OK;
  if (!amps || !out_idx || !out_prob) return set_error(LF_INVALID_ARGUMENT, "NULL pointer");
  if (reinterpret_cast<uintptr_t>(amps) % 16 != 0)
    return set_error(LF_INVALID_ARGUMENT, "amps must be 16-byte aligned");
  if (group_size < 1 || group_size > (int64_t(1) << 40))
    return set_error(LF_INVALID_ARGUMENT, "group_size out of range");
  if (n_groups > (int64_t(1) << 40) / group_size)
    return set_error(LF_INVALID_ARGUMENT, "n_groups * group_size above 2^40");
  if (k < 1 || k > group_size) return set_error(LF_INVALID_ARGUMENT, "k out of range");
  if (int64_t(k) * n_groups > (int64_t(1) << 31))
    return set_error(LF_INVALID_ARGUMENT, "n_groups * k above 2^31");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const double* a = static_cast<const double*>(amps);
  if (!lf::select_uses_radix(group_size, k)) {
    hipError_t e = lf::launch_topk(a, n_groups, group_size, k, out_idx, out_prob, st);
    if (e != hipSuccess) return set_error(LF_HIP_ERROR, std::string("top-k launch: ") + hipGetErrorString(e));
    return LF_OK;
  }
  if (lf::select_scratch_bytes(k) > lf::NOALLOC_SCRATCH_BYTES)
    return set_error(LF_INVALID_ARGUMENT, "k needs more than the fixed " +
                                              std::to_string(lf::NOALLOC_SCRATCH_BYTES >> 20) +
                                              " MiB of scratch of lf_postselect_topk_noalloc (k <= " +
                                              std::to_string(lf::noalloc_max_k()) + ")");
  void* scratch = nullptr;
  lf_status r = lf::noalloc_scratch(&scratch);
  if (r != LF_OK) return r;
  hipError_t e = lf::launch_select(a, n_groups, group_size, k, out_idx, out_prob, scratch, st);
  if (e != hipSuccess) return set_error(LF_HIP_ERROR, std::string("top-k selection: ") + hipGetErrorString(e));
  return LF_OK;
}

lf_status lf_probabilities_at(const void* amps, int64_t n, const int64_t* idx, int64_t m, double* out_prob,
                              void* stream) {
  if (m < 0 || n < 0) return set_error(LF_INVALID_ARGUMENT, "negative size");
  if (m == 0) return LF_OK;
  if (!amps || !idx || !out_prob) return set_error(LF_INVALID_ARGUMENT, "NULL pointer");
  const int64_t blocks = (m + 255) / 256;
  if (blocks > 0x7fffffff) return set_error(LF_INVALID_ARGUMENT, "m too large");
  hipLaunchKernelGGL(lf::probs_at_kernel, dim3(unsigned(blocks)), dim3(256), 0, static_cast<hipStream_t>(stream),
                     static_cast<const double*>(amps), n, idx, m, out_prob);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(LF_HIP_ERROR, std::string("probabilities: ") + hipGetErrorString(e));
  return LF_OK;
}

}  // extern "C"
