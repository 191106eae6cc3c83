// MCMC sampling from approximate probabilities: the baseline that the
// top-k post-selection is compared with (Methods B).  Samples drawn from the
// approximate p of a fraction-f contraction have an XEB close to f (Eq. 3);
// top-k selection raises it by about ln(|S~|/k) (Eq. 4).
//
// Independence Metropolis-Hastings over a structured candidate set S~
// (groups of correlated strings): every chain proposes a candidate uniformly
// from S~ and moves there with probability min(1, p_new / p_cur), so its
// stationary distribution is p restricted to S~, normalised.  One thread per
// chain; after `burn_in` moves every `thin`-th state is a sample.
//
// Random numbers: each chain runs its own SplitMix64 sequence (Steele, Lea
// and Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014):
// state += 0x9E3779B97F4A7C15, output = the published 64-bit finaliser of the
// state; the chain's starting state is that finaliser applied to
// seed + (chain + 1) * 0x9E3779B97F4A7C15.  A candidate is the high 64 bits
// of output * |S~| (uniform up to 2^-64 relative bias); an acceptance uniform
// is the top 53 bits of an output times 2^-53.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/leapfrog.h"
#include "kernels.h"

namespace lf {

lf_status set_error(lf_status s, const std::string& msg);  // runtime.hip

namespace {

constexpr uint64_t SM64_GAMMA = 0x9E3779B97F4A7C15ull;

__device__ __forceinline__ uint64_t sm64_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void __launch_bounds__(256) mcmc_kernel(const double* amps, int64_t n_amps, const int64_t* base,
                                                   int64_t group_size, int64_t stride, uint64_t n_cand,
                                                   int64_t n_chains, int64_t burn_in, int64_t thin,
                                                   int64_t per_chain, uint64_t seed, int64_t* out,
                                                   int64_t* accepted) {
  const int64_t c = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (c >= n_chains) return;
  uint64_t state = sm64_mix(seed + SM64_GAMMA * (uint64_t(c) + 1));
  auto next = [&]() {
    state += SM64_GAMMA;
    return sm64_mix(state);
  };
  auto pos_of = [&](uint64_t ci) {
    return base[ci / uint64_t(group_size)] + int64_t(ci % uint64_t(group_size)) * stride;
  };
  auto p_at = [&](int64_t pos) {
    if (pos < 0 || pos >= n_amps) return 0.0;
    return prob_of(amps[2 * pos], amps[2 * pos + 1]);
  };
  int64_t cur = pos_of(__umul64hi(next(), n_cand));
  double cur_p = p_at(cur);
  int64_t acc = 0, emitted = 0;
  const int64_t total = burn_in + per_chain * thin;
  for (int64_t t = 1; t <= total; ++t) {
    const int64_t cand = pos_of(__umul64hi(next(), n_cand));
    const double cp = p_at(cand);
    const double u = double(next() >> 11) * 0x1.0p-53;
    if (u * cur_p < cp) {
      cur = cand;
      cur_p = cp;
      ++acc;
    }
    if (t > burn_in && (t - burn_in) % thin == 0) out[c * per_chain + emitted++] = cur;
  }
  accepted[c] = acc;
}

}  // namespace
}  // namespace lf

extern "C" lf_status lf_mcmc_sample(const void* amps, int64_t n_amps, const int64_t* group_base,
                                    int64_t n_groups, int64_t group_size, int64_t stride, int64_t n_chains,
                                    int64_t burn_in, int64_t thin, int64_t per_chain, uint64_t seed,
                                    int64_t* out_pos, int64_t* out_accepted, void* stream) {
  if (!amps || !group_base || !out_pos || !out_accepted) return lf::set_error(LF_INVALID_ARGUMENT, "NULL pointer");
  if (n_amps < 1 || n_groups < 1 || group_size < 1 || n_chains < 1 || burn_in < 0 || thin < 1 || per_chain < 1)
    return lf::set_error(LF_INVALID_ARGUMENT, "sizes must be positive (burn_in >= 0)");
  if (n_groups > (int64_t(1) << 62) / group_size) return lf::set_error(LF_INVALID_ARGUMENT, "too many candidates");
  if (per_chain > (int64_t(1) << 40) / n_chains || thin > (int64_t(1) << 40) / per_chain)
    return lf::set_error(LF_INVALID_ARGUMENT, "chain length or sample count too large");
  const int64_t blocks = (n_chains + 255) / 256;
  if (blocks > 0x7fffffff) return lf::set_error(LF_INVALID_ARGUMENT, "too many chains");
  hipLaunchKernelGGL(lf::mcmc_kernel, dim3(unsigned(blocks)), dim3(256), 0, static_cast<hipStream_t>(stream),
                     static_cast<const double*>(amps), n_amps, group_base, group_size, stride,
                     uint64_t(n_groups) * uint64_t(group_size), n_chains, burn_in, thin, per_chain, seed,
                     out_pos, out_accepted);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return lf::set_error(LF_HIP_ERROR, std::string("mcmc launch: ") + hipGetErrorString(e));
  return LF_OK;
}
