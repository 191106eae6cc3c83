/*
 * leapfrog.h - C ABI of the sliced tensor-network amplitude library for
 * MI355X (gfx950).
 *
 * The method (arXiv 2406.18889, Methods A and C): the amplitudes of a random
 * quantum circuit for k groups of 2^l correlated bitstrings (l open output
 * qubits take all values; the other qubits are fixed to k sampled closed
 * strings) are computed by contracting the circuit's tensor network.  The
 * network is sliced: a set of S wires is fixed to each of its 2^S value
 * combinations, every combination (a slice, or sub-network) is contracted
 * independently, and the network's value is the sum over all slices
 * (slicing identity, Methods C).  Summing only a fraction f of the slices
 * gives an approximation whose fidelity is close to f (Eq. 3).  The top-k
 * step (Methods A and B, Eq. 2, Appendix A) then keeps, per group or over
 * all groups, the k strings with the largest |amplitude|^2.
 *
 * Conventions
 *  - Basis: qubit 0 is the least significant bit of a basis index.  A
 *    two-qubit gate matrix is indexed by 2*bit(q[0]) + bit(q[1]); row =
 *    output.  Matrices are complex128, row-major, (re, im) interleaved.
 *  - Output amplitudes: out[b * 2^l + j] is the amplitude of closed string b
 *    with bit open_qubits[i] of the result equal to bit i of j.
 *  - A wire (q, j), 1 <= j < number of two-qubit gates on q, is the point
 *    on qubit q immediately before its j-th (0-based) two-qubit gate, after
 *    the single-qubit gates that precede it.  Sliced wire t takes bit t of
 *    the slice number, so the slice prefix [0, 2^(S-D)) fixes the D
 *    last-listed sliced wires to 0.
 *  - Every call returns an lf_status; 0 is success.  No exception crosses
 *    the boundary.  lf_last_error() returns a thread-local message for the
 *    last failing call on the calling thread.
 *  - Device pointers are HIP device addresses owned by the caller; `stream`
 *    is a hipStream_t (NULL = the default stream).  Calls that take a stream
 *    are asynchronous on it unless stated otherwise.
 */
#ifndef LEAPFROG_H
#define LEAPFROG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lf_status;
enum {
  LF_OK = 0,
  LF_INVALID_ARGUMENT = 1, /* malformed circuit, qubit list, range or size */
  LF_PLAN_INFEASIBLE = 2,  /* no tree fits the cap within 64 sliced wires */
  LF_OUT_OF_WORKSPACE = 3, /* bound workspace smaller than required */
  LF_HIP_ERROR = 4,        /* a HIP runtime call failed */
  LF_OVERFLOW = 5,         /* complex-half saturation in the contracted range */
  LF_NOT_BOUND = 6,        /* contraction before lf_plan_bind_workspace */
  LF_INTERNAL = 7
};

enum { LF_C64 = 0, LF_CHALF = 1 };          /* contraction arithmetic */
enum { LF_COST_FLOPMEM = 0, LF_COST_MLP = 1 }; /* path-search cost model */
enum { LF_LAUNCH_STREAM = 0, LF_LAUNCH_GRAPH = 1 };
enum { LF_OVERFLOW_RECALIBRATE = 0, LF_OVERFLOW_REPORT = 1 }; /* complex-half saturation policy */
enum { LF_MULT_AUTO = 0, LF_MULT_4M = 1, LF_MULT_3M = 2 };    /* real products per complex product */

typedef struct lf_gate {
  int32_t n_q;       /* 1 or 2 */
  int32_t q[2];      /* qubits; q[1] unused for n_q == 1 */
  int32_t layer;     /* cycle index (informational) */
  double mat[32];    /* (re, im) pairs, row-major 2x2 (first 8) or 4x4 */
} lf_gate;

typedef struct lf_circuit {
  int32_t n_qubits;  /* 1..63 */
  int32_t n_gates;
  const lf_gate* gates; /* in time order */
} lf_circuit;

typedef struct lf_plan_opts {
  int32_t dtype;                 /* LF_C64 or LF_CHALF */
  int32_t max_log2_intermediate; /* cap M: every sliced intermediate <= 2^M elements */
  int32_t n_sliced_wires;        /* -1: as many as the cap needs; >= 0: at least this many */
  const int32_t* sliced_wires;   /* optional forced wires, pairs (q, j), bit order; NULL = planner */
  int32_t n_forced;              /* number of pairs in sliced_wires */
  int32_t cost_model;            /* LF_COST_FLOPMEM or LF_COST_MLP (needs a loaded model):
                                    the cost that ranks the refined candidates (restarts) */
  int32_t greedy_trials;         /* randomized greedy trees tried */
  int32_t partition_trials;      /* recursive min-cut bisection trees tried */
  int64_t sa_iters;              /* annealing moves over the best tree (0 = none) */
  uint64_t seed;                 /* search seed */
  int32_t chalf_min_log2;        /* complex-half only: steps touching a tensor of at
                                    least 2^this elements run in half, smaller ones in
                                    complex64 */
  int32_t launch_mode;           /* LF_LAUNCH_STREAM or LF_LAUNCH_GRAPH */
  int32_t check_overflow;        /* nonzero: lf_contract_slices synchronizes at its end
                                    and handles saturation by overflow_policy */
  int32_t slices_per_graph;      /* graph mode: slices captured per graph replay */
  int32_t search_dtype;          /* arithmetic whose step costs the search minimises;
                                    -1 = dtype.  Two plans that differ only in dtype and
                                    share search_dtype get the same tree and slices */
  int32_t autotune;              /* nonzero: the first contraction times every applicable
                                    kernel variant (tile shape) per step shape and keeps
                                    the fastest; results are shared by the process */
  int32_t restarts;              /* >= 1: the `restarts` best candidate trees are each
                                    annealed and sliced to the cap; the ranking cost
                                    (cost_model: the learned model, else FLOP + memory)
                                    of the whole sliced network picks one.  The search
                                    itself (trees, annealing, sliced wires) always runs
                                    on FLOP + memory */
  int32_t chalf_headroom_bits;   /* complex-half: the shift of each step is calibrated so
                                    the largest |re|,|im| of its result on the calibration
                                    slice is at most 2^(16 - this); in [-8, 24], default 4 */
  int32_t overflow_policy;       /* with check_overflow: LF_OVERFLOW_RECALIBRATE (default)
                                    re-derives the shifts on the first saturated slice with
                                    two more bits of headroom and contracts the rest of the
                                    range again (at most 3 times per call);
                                    LF_OVERFLOW_REPORT returns LF_OVERFLOW at once */
  int32_t chalf_exec_min_log2;   /* complex-half: the threshold of chalf_min_log2 for the
                                    execution only (-1 = chalf_min_log2).  The search still
                                    costs steps with chalf_min_log2, so plans that differ
                                    only here share their tree and slices while more (or
                                    fewer) steps run in complex64 */
  int32_t mult;                  /* LF_MULT_AUTO or LF_MULT_4M: every complex product is
                                    four real products on MFMA (the real and imaginary
                                    parts of C as two real GEMMs over 2K against operand
                                    forms of B made in registers).  LF_MULT_3M is
                                    rejected (LF_INVALID_ARGUMENT): it would need the sums
                                    Ar + Ai and Br + Bi as extra operand tensors and loses
                                    bits to cancellation in complex-half */
  const char* autotune_cache;    /* NULL, or a file of kernel choices (lf_autotune_save
                                    format): merged into the process's choices when the
                                    plan is built (if the file exists) and rewritten with
                                    them after the plan's first contraction has tuned */
  int32_t keep_batch_order;      /* 0 (default): the library contracts the closed strings
                                    in its own order, sorted by the closed bits that select
                                    the blocks of gathered operands (strings that share a
                                    block become neighbours, so its reads hit in cache);
                                    out_amps rows stay in the caller's order.  1: contract
                                    them in the given order */
  int32_t group_small_steps;     /* 1 (default): consecutive small independent steps that
                                    run on the streaming kernel go out as one launch
                                    (results identical); 0: one launch per step */
} lf_plan_opts;

typedef struct lf_plan_info {
  int64_t n_slices;              /* 2^S */
  int32_t n_sliced_wires;        /* S */
  int32_t n_steps;               /* pairwise contractions */
  int32_t n_variant_steps;       /* steps that depend on the slice */
  int32_t n_leaves;
  int32_t max_log2_intermediate; /* largest tensor of one slice, log2 elements */
  int32_t dtype;
  int32_t n_open;
  int64_t n_batch;
  int32_t n_batch_log2;          /* batch padded to 2^this */
  int32_t n_half_steps;          /* steps computed in complex-half */
  double macs_per_slice;         /* complex multiply-adds of the slice-dependent steps */
  double macs_invariant;         /* once per plan: slice-independent subtrees */
  double bytes_per_slice;        /* operand + result bytes of the slice-dependent steps */
  double bytes_invariant;
  double log2_total_macs;        /* all slices */
  uint64_t workspace_bytes;      /* device bytes lf_plan_bind_workspace needs */
  int32_t leaf_id_base;          /* first node id of an intermediate in lf_plan_tree */
  int32_t n_step_groups;         /* launches that each run several small slice-dependent
                                    steps (group_small_steps), as set up by the last
                                    contraction; 0 before the first one */
  int32_t n_grouped_steps;       /* the steps in them */
} lf_plan_info;

typedef struct lf_plan lf_plan;

/* Defaults: LF_C64, cap 2^28, planner-chosen slices, FLOP+memory cost,
 * 8 greedy and 64 partition trials, no annealing, seed 1, chalf_min_log2 16,
 * stream launch, autotuning on, overflow check on with recalibration,
 * 4 bits of complex-half headroom, 8 slices per graph, 1 restart. */
void lf_plan_opts_default(lf_plan_opts* opts);

/*
 * Builds the network of `circuit` with output qubits `open_qubits` (l of
 * them, l <= 30) and `n_batch` closed strings `closed_bits` (each a full
 * n-bit mask; bits at open positions are ignored; n_batch <= 2^22, padded
 * internally to a power of two), folds single-qubit gates in float64,
 * searches a contraction tree and slicing under the cap (Methods C, D), lays
 * out every tensor (dimension order, Methods C) and returns an opaque plan
 * in *out_plan, owned by the caller and freed with lf_plan_destroy.  Host
 * only; no device call.  Errors: LF_INVALID_ARGUMENT, LF_PLAN_INFEASIBLE.
 */
lf_status lf_build_network(const lf_circuit* circuit, const int32_t* open_qubits,
                           int32_t n_open, const uint64_t* closed_bits, int64_t n_batch,
                           const lf_plan_opts* opts, lf_plan** out_plan);

lf_status lf_plan_get_info(const lf_plan* plan, lf_plan_info* out);

/* Sliced wires as pairs (q, j) in bit order: out_qj[2t], out_qj[2t+1]. */
lf_status lf_plan_sliced_wires(const lf_plan* plan, int32_t* out_qj);

/*
 * The contraction tree: leaf_canon[i] is the canonical id of leaf node i
 * (the k-th two-qubit gate of the circuit is leaf k; a qubit q without a
 * two-qubit gate is leaf n_2q + q); step s contracts nodes left[s] and
 * right[s], given as canonical leaf ids or as leaf_id_base + s' for the
 * result of an earlier step s'.  Steps are in execution order.
 */
lf_status lf_plan_tree(const lf_plan* plan, int32_t* leaf_canon, int32_t* left, int32_t* right);

/*
 * Per-step shape: dims[8s .. 8s+7] = (nz, nm, nn, nk, variant, dtype,
 * out_dtype, kernel) where the step computes C[z,m,n] = sum_k A[z,m,k] B[z,n,k]
 * over 2^nz x 2^nm x 2^nn x 2^nk; macs[s], bytes[s] its work.  Either
 * output pointer except dims may be NULL.
 */
lf_status lf_plan_steps(const lf_plan* plan, int32_t* dims, double* macs, double* bytes);

/* Result strides of step s (elements): out[0..nz) for the bits of z, then
 * nm for m, then nn for n, as in lf_contract_pair; out must hold nz+nm+nn. */
lf_status lf_plan_step_strides(const lf_plan* plan, int32_t step, int64_t* out);

/*
 * Operands of a batched step (Methods C, sparse final stem stages): for
 * operand A (w = 0) and B (w = 1), info[3w] = 1 if the operand is stored per
 * batch entry (the running batched tensor), 0 if it is a plain tensor whose
 * block for closed string b is chosen by the bits of b at its closed qubits,
 * -1 if the step is not batched; info[3w + 1] = the number of those qubits
 * (at most 64), written to qa / qb (either may be NULL) with their element
 * strides in sa / sb (either may be NULL).  info must hold 6 values.
 */
lf_status lf_plan_step_gather(const lf_plan* plan, int32_t step, int32_t* info, int32_t* qa, int64_t* sa,
                              int32_t* qb, int64_t* sb);

/*
 * Binds `bytes` of device memory at `dev_ptr` (256-byte aligned, owned by
 * the caller, at least info.workspace_bytes) and uploads the leaf tensors on
 * `stream`.  The workspace must stay valid until the plan is destroyed or
 * rebound.  Errors: LF_OUT_OF_WORKSPACE, LF_INVALID_ARGUMENT, LF_HIP_ERROR.
 */
lf_status lf_plan_bind_workspace(lf_plan* plan, void* dev_ptr, uint64_t bytes, void* stream);

/*
 * Contracts slices [slice_begin, slice_end) and ADDS their sum to
 * out_amps (device, complex128, [n_batch][2^l], (re, im) interleaved,
 * 16-byte aligned, else LF_INVALID_ARGUMENT), in float64, one slice after another in increasing order (deterministic).
 * The full range gives the exact amplitudes; a prefix gives the fraction f
 * of Methods A.  begin == end is a no-op.  A plan is used by one stream at a
 * time.
 *
 * Complex-half saturation (an extension; the paper computes in complex64):
 * a slice in which any value had to be clamped to the half range, and every
 * slice after it, is NOT added: out_amps always holds the sum of the slices
 * before the first saturated one, whose number the plan records (see
 * lf_plan_overflow; the state persists until cleared).  Without
 * check_overflow the call is asynchronous and the caller reads that state
 * itself.  With check_overflow the call synchronizes; on saturation the
 * LF_OVERFLOW_RECALIBRATE policy re-derives the shifts on the first
 * saturated slice (two more bits of headroom) and contracts the rest of the
 * range again, so the call returns LF_OK with every slice added; after 3
 * such attempts, or under LF_OVERFLOW_REPORT, it returns LF_OVERFLOW with
 * out_amps holding the slices before lf_overflow_info.first_bad_slice.
 * Errors: LF_NOT_BOUND, LF_INVALID_ARGUMENT, LF_HIP_ERROR, LF_OVERFLOW.
 */
lf_status lf_contract_slices(lf_plan* plan, int64_t slice_begin, int64_t slice_end,
                             void* out_amps, void* stream);

/* Saturation state of a complex-half plan (complex64 plans read zeros). */
typedef struct lf_overflow_info {
  uint32_t saturated;        /* values clamped to the half range since the last clear */
  int32_t recalibrations;    /* automatic recalibrations since the workspace was bound */
  int64_t first_bad_slice;   /* first slice left out of an accumulator; -1 = none */
  int32_t headroom_bits;     /* current calibration headroom (see lf_plan_opts) */
  int32_t reserved;
} lf_overflow_info;

/* Reads the saturation state into *out (synchronizes `stream`) and, if
 * `clear` is nonzero, resets the counter and the recorded slice so later
 * slices are added again.  Errors: LF_INVALID_ARGUMENT, LF_NOT_BOUND,
 * LF_HIP_ERROR. */
lf_status lf_plan_overflow(lf_plan* plan, void* stream, lf_overflow_info* out, int32_t clear);

/* Re-derives the complex-half shift of every step from slice `sigma` with
 * `headroom_bits` bits of headroom (the largest |re|,|im| of each step's
 * result on that slice becomes at most 2^(16 - headroom_bits)), recomputes
 * the slice-independent results with them and clears the saturation state.
 * A no-op for complex64 plans.  Synchronous.  Errors: LF_INVALID_ARGUMENT,
 * LF_NOT_BOUND, LF_HIP_ERROR. */
lf_status lf_plan_recalibrate(lf_plan* plan, int64_t sigma, int32_t headroom_bits, void* stream);

/* Fault injection for tests of the saturation handling (no use in a
 * computation): multiplies, in the workspace, the entries of the first leaf
 * that carries sliced wire `wire_bit` whose value of that wire is `value` by
 * 2^log2_factor, without changing the leaf's recorded exponent, so slices
 * with bit wire_bit == value carry values 2^log2_factor larger than the
 * calibration saw.  log2_factor 0 restores the leaf.  Synchronous.  Errors:
 * LF_INVALID_ARGUMENT (ranges; a complex-half leaf pushed outside the half
 * range), LF_NOT_BOUND, LF_HIP_ERROR. */
lf_status lf_debug_scale_slice_leaf(lf_plan* plan, int32_t wire_bit, int32_t value,
                                    int32_t log2_factor, void* stream);

/*
 * Batched execution of many sliced subtasks of uneven shape.  Item i adds
 * slices [slice_begin, slice_end) of items[i].plan into items[i].out_amps,
 * exactly as lf_contract_slices would.  Items of the same plan run in item
 * order (they share that plan's workspace); items of different plans are
 * independent.  mode LF_BATCH_SEQUENTIAL launches every item's kernels on
 * `stream` in item order.  LF_BATCH_GRAPH groups the items into one chain
 * per plan, deals the chains to `lanes` lanes by their work (slices times
 * the plan's time per slice, measured once per plan on `stream` the first
 * time it is batched, without touching any accumulator; heaviest first onto
 * the least loaded lane; 1..8, 0 = one lane per plan up to 4), records each
 * lane once as a HIP
 * graph, and on every call forks the lanes from `stream`, launches one graph
 * per lane on a library-owned stream of its own and joins them back into
 * `stream` (so different plans run concurrently); the recorded graphs are
 * reused while the items are unchanged (and the plans have not been rebound
 * or recalibrated since).  Every plan must be bound.  Results are
 * bit-identical between the modes.  Saturation gating is as in
 * lf_contract_slices (per plan, in item order); without recalibration: if
 * any item's plan has check_overflow set, the call synchronizes at its end
 * and returns LF_OVERFLOW when such a plan saturated.  Otherwise
 * asynchronous.  Errors: as lf_contract_slices.
 */
typedef struct lf_batch_item {
  lf_plan* plan;
  int64_t slice_begin, slice_end;
  void* out_amps;
} lf_batch_item;
enum { LF_BATCH_SEQUENTIAL = 0, LF_BATCH_GRAPH = 1 };
lf_status lf_contract_batch(const lf_batch_item* items, int32_t n_items, int32_t mode,
                            int32_t lanes, void* stream);

/*
 * Top-k post-selection (Methods A): for each of n_groups consecutive groups
 * of group_size complex128 amplitudes, p = re*re + im*im in float64 (each
 * product and the sum rounded separately), ordered by p descending then
 * position ascending; writes the first k positions to out_idx[g*k + r]
 * (int64, device) and their p to out_prob (float64, device).  group_size =
 * 2^l gives one selection per closed string; group_size = n_batch * 2^l
 * selects over all candidates (the paper's global top-k over S~).  Limits:
 * 1 <= k <= group_size, n_groups * group_size <= 2^40, n_groups * k <= 2^31;
 * amps 16-byte aligned.  Small selections (group_size <= 2^16 and k <= 1024)
 * run one workgroup per group and are asynchronous.  Larger ones select
 * with device-side radix selection over the bit patterns of p (p >= 0 orders
 * as its bits do), an ordered compaction and a stable radix sort, group after
 * group; they use device scratch of about 16 k bytes + 100 KiB that this
 * call allocates and frees, so they synchronize `stream`.  The result is the
 * same either way.  p of a NaN amplitude is unordered: its position in the
 * result is unspecified.  Errors: LF_INVALID_ARGUMENT, LF_HIP_ERROR.
 */
lf_status lf_postselect_topk(const void* amps, int64_t n_groups, int64_t group_size, int32_t k,
                             int64_t* out_idx, double* out_prob, void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * selection, arguments and result as lf_postselect_topk, but the large-size
 * path keeps its scratch in a fixed 64 MiB device array that the library
 * holds on each GPU it runs on until the process ends, so the call allocates
 * nothing and is asynchronous on `stream` in every case.  Limit: k <= about
 * 4.17 million (scratch of about 16.06 k bytes + 97 KiB); a larger k returns
 * LF_INVALID_ARGUMENT.  Every call on one GPU shares that GPU's array:
 * calls that may overlap in time on one GPU (different streams, threads)
 * race and must be serialized by the caller.  Errors: LF_INVALID_ARGUMENT,
 * LF_HIP_ERROR.
 */
lf_status lf_postselect_topk_noalloc(const void* amps, int64_t n_groups, int64_t group_size,
                                     int32_t k, int64_t* out_idx, double* out_prob, void* stream);

/*
 * p of selected amplitudes, for the cross-entropy benchmark of a selection
 * (Methods B, Eq. 1: XEB = N/|S| sum over S of q - 1, with q the ideal
 * probabilities): out_prob[r] = re*re + im*im (float64, no fused rounding) of
 * element idx[r] of the n complex128 amplitudes at amps (device), NaN where
 * idx[r] is outside [0, n).  All pointers device memory; asynchronous.
 * Errors: LF_INVALID_ARGUMENT, LF_HIP_ERROR.
 */
lf_status lf_probabilities_at(const void* amps, int64_t n, const int64_t* idx, int64_t m,
                              double* out_prob, void* stream);

/*
 * Sampling baseline of Methods B (Eq. 3: samples drawn from the approximate
 * p of a fraction-f contraction have XEB close to f): n_chains independent
 * Metropolis chains over the candidate set S~ = {group_base[g] + j * stride :
 * g < n_groups, j < group_size} of positions in the n_amps complex128
 * amplitudes at amps (device).  Each chain proposes a uniform candidate and
 * moves with probability min(1, p_new / p_cur), p = re*re + im*im (float64,
 * no fused rounding; 0 outside [0, n_amps)); after burn_in moves it writes
 * every thin-th position to out_pos[chain * per_chain + i] (int64 device,
 * n_chains * per_chain) and its accepted moves to out_accepted[chain].
 * Random numbers: one SplitMix64 sequence per chain from `seed`.  group_base
 * is an int64 device array.  Asynchronous.  Errors: LF_INVALID_ARGUMENT,
 * LF_HIP_ERROR.
 */
lf_status lf_mcmc_sample(const void* amps, int64_t n_amps, const int64_t* group_base, int64_t n_groups,
                         int64_t group_size, int64_t stride, int64_t n_chains, int64_t burn_in,
                         int64_t thin, int64_t per_chain, uint64_t seed, int64_t* out_pos,
                         int64_t* out_accepted, void* stream);

/*
 * Times every step of slice 0 on `stream` with HIP events (reps runs each,
 * after one warm-up) and writes the mean milliseconds per step to out_ms
 * [n_steps].  Synchronous.  Needs a bound workspace.
 */
lf_status lf_profile_steps(lf_plan* plan, int32_t reps, double* out_ms, void* stream);

/*
 * Live timing of one contraction kernel inside lf_contract_slices (not a
 * step of the method: instrumentation for measuring the steps where they
 * run).  After lf_plan_time_kernel(plan, kernel, reserve), every launch of
 * the steps whose kernel id (dims[7] of lf_plan_steps) equals `kernel` is
 * bracketed by a pair of HIP events on the caller's stream, in stream launch
 * mode only (graph launches are not timed).  `reserve` pre-creates events
 * for that many launches so that none is created while timing; more are
 * created on demand.  kernel -1 switches timing off.  Errors:
 * LF_INVALID_ARGUMENT (kernel id, reserve outside [0, 2^20]), LF_HIP_ERROR.
 *
 * lf_plan_kernel_times waits for the last timed launch and returns the
 * milliseconds summed over the launches timed since the previous call and
 * their count; per_step_ms and per_step_launches (nullable host arrays of
 * n_steps) receive the same per step.  The counters then restart.
 */
lf_status lf_plan_time_kernel(lf_plan* plan, int32_t kernel, int64_t reserve);
lf_status lf_plan_kernel_times(lf_plan* plan, double* total_ms, int64_t* launches,
                               double* per_step_ms, int64_t* per_step_launches);

/*
 * One pairwise complex contraction, the operation every step of a plan
 * performs (Methods C):  C[z,m,n] = scale * sum_k A[z,m,k] * B[z,n,k]  over
 * 2^nz x 2^nm x 2^nn x 2^nk.  A is a row-major [2^nz][2^nm][2^nk] array of
 * (re, im) pairs in dtype_a and B a row-major [2^nz][2^nn][2^nk] array in
 * dtype_b (equal, or a complex-half A with a complex64 B); C
 * element (z,m,n) is written, in dtype_out, at element offset
 * sum_b bit_b(z) c_strides[b] + sum_b bit_b(m) c_strides[nz+b] +
 * sum_b bit_b(n) c_strides[nz+nm+b]; the strides must map distinct (z,m,n)
 * to distinct elements.  kernel: 0 streaming (one row per thread), 1 MFMA
 * 128 x 64 complex tile, 2 MFMA 256 x 64 tile (complex-half), 3 streaming
 * with B staged in LDS (2^nn 2^nk <= 256, 2^nm >= 256), 4 MFMA 256 x 128
 * tile (complex-half), 5 the 256 x 128 tile with double-buffered LDS
 * (complex-half), 6 the 256 x 128 tile with 64-deep K steps (complex-half),
 * 7 MFMA on 32-row groups against a B of 2^nn <= 16 rows held in registers
 * (complex-half A, 2 <= nk <= 6), 8, 9 and 10 kernels 2, 5 and 4 with tiles
 * dealt to the XCDs in contiguous groups, 11 the 256 x 128 tile on eight
 * waves with operands loaded straight into a three-stage LDS ring
 * (complex-half, 2^nm a multiple of 256, 2^nn of 128, 5 <= nk <= 21), 12
 * kernel 11 with the XCD-grouped tile order, 13 and 14 kernels 11 and 12 on
 * four waves (one per SIMD), 15 one sixteen-wave workgroup per batch entry
 * with K split over the waves (complex-half, nm <= 5, nn <= 5, nk >= 7),
 * 16 and 17 the 128 x 128 tile of kernel 11 on four waves with two operand
 * stages, two workgroups per CU (complex-half, 2^nm and 2^nn multiples of
 * 128, 5 <= nk <= 21), in the two tile orders, -1 the default choice; a kernel that does
 * not apply to the
 * shape or dtype falls back to 0.  Device pointers owned by the caller; A and
 * B 16-byte aligned.  Limits: nz <= 20, nm, nn <= 40.  Errors:
 * LF_INVALID_ARGUMENT, LF_HIP_ERROR.
 */
lf_status lf_contract_pair(int32_t dtype_a, int32_t dtype_b, int32_t dtype_out, int32_t kernel,
                           const void* A, const void* B, void* C, int32_t nz, int32_t nm, int32_t nn,
                           int32_t nk, const int64_t* c_strides, float scale, void* stream);

/* ------------------------------------------------------------------------
 * Learned step-cost model (planner extension): a three-layer perceptron
 * in -> H -> H -> 1 with ReLU on both hidden layers, float32, regressing the
 * log of a contraction step's run time from LF_N_FEATURES features of the
 * step's shape; fitted by mean squared error with Adam.  The parameters are
 * one float32 device array: W1 [in][H] row-major, b1 [H], W2 [H][H], b2 [H],
 * W3 [H], b3 [1].  All arrays here are caller-owned device memory.
 * ---------------------------------------------------------------------- */
#define LF_N_FEATURES 14

/* Features of a step over 2^nz x 2^nm x 2^nn x 2^nk (see lf_plan_steps) in
 * arithmetic dtype: nz, nm, nn, nk, log2 of multiply-adds, log2 sizes of A,
 * B and C, log2 bytes, log2 arithmetic intensity, dtype, MFMA-tile flag,
 * batched flag, log2 roofline microseconds.  Host only.  out[LF_N_FEATURES]. */
lf_status lf_step_features(int32_t nz, int32_t nm, int32_t nn, int32_t nk, int32_t dtype,
                           float* out);

/* Parameter count and workspace bytes for batches up to max_batch. */
lf_status lf_mlp_sizes(int32_t n_in, int32_t hidden, int64_t max_batch, int64_t* n_params,
                       uint64_t* workspace_bytes);

/* Y[batch] = network(X[batch][n_in]).  Asynchronous on stream. */
lf_status lf_mlp_forward(const float* params, int32_t n_in, int32_t hidden, const float* X,
                         int64_t batch, float* Y, void* workspace, uint64_t workspace_bytes,
                         void* stream);

/* loss[0] = mean((Y - T)^2) and grads[n_params] = its gradient (same layout
 * as params), for one batch.  Asynchronous on stream. */
lf_status lf_mlp_gradients(const float* params, int32_t n_in, int32_t hidden, const float* X,
                           const float* T, int64_t batch, float* grads, float* loss,
                           void* workspace, uint64_t workspace_bytes, void* stream);

/* One Adam update (step counts from 1) of params with moments m, v. */
lf_status lf_mlp_adam_step(float* params, float* m, float* v, const float* grads, int64_t n_params,
                           int32_t step, float lr, float beta1, float beta2, float eps, void* stream);

/*
 * Trains the network on the GPU with the library's own kernels (the
 * extension's learned part): X [n][n_in] and T [n] are host arrays of raw
 * features and targets (log seconds); they are standardised (population
 * mean and deviation, written to x_mean [n_in], x_std [n_in], y_mean,
 * y_std, host) and the parameters (device, [lf_mlp_sizes n_params],
 * initialised by the caller) are fitted by mean squared error with Adam
 * (beta 0.9, 0.999, eps 1e-8), `epochs` passes over a seeded shuffle in
 * batches of `batch` rows (a last partial batch is dropped), learning rate
 * lr * (1 + cos(pi epoch / epochs)) / 2.  curve (host [epochs], nullable)
 * receives the mean batch loss per epoch.  Device temporaries are allocated
 * and freed inside; synchronous on stream.  Errors: LF_INVALID_ARGUMENT,
 * LF_HIP_ERROR.
 */
lf_status lf_costmodel_train(const float* X, const float* T, int64_t n, int32_t n_in, int32_t hidden,
                             int32_t epochs, int32_t batch, float lr, uint64_t seed, float* params,
                             float* x_mean, float* x_std, float* y_mean, float* y_std, float* curve,
                             void* stream);

/* Loads a trained network (host copy of params, n_in == LF_N_FEATURES) with
 * its feature standardisation (x - x_mean[i]) / x_std[i] and target
 * log(seconds) = y * y_std + y_mean, for plans built with LF_COST_MLP.  Such
 * plans evaluate it on the current device with lf_mlp_forward, once per
 * batch exponent, over every step shape the search can meet (a host table
 * of predicted seconds); lf_build_network then needs a GPU. */
lf_status lf_costmodel_load(const float* params, int32_t n_in, int32_t hidden, const float* x_mean,
                            const float* x_std, float y_mean, float y_std);
lf_status lf_costmodel_clear(void);

/* Predicted seconds of one step under the loaded model (tabulates on first
 * use of nz).  Errors: LF_INVALID_ARGUMENT when no model is loaded. */
lf_status lf_costmodel_predict(int32_t nz, int32_t nm, int32_t nn, int32_t nk, int32_t dtype,
                               double* seconds);

/* The autotuner's choices (step shape and operand types -> kernel variant)
 * are shared by all plans of the process; these save them to a text file
 * and merge them back, so a later process skips the timing runs. */
lf_status lf_autotune_save(const char* path);
lf_status lf_autotune_load(const char* path);

void lf_plan_destroy(lf_plan* plan);

const char* lf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LEAPFROG_H */
