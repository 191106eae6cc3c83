/*
 * Oracle (test infrastructure only): plain complex128 state-vector simulator.
 *
 * What the path computes, by its definition: psi = U|0...0>, with U the
 * circuit of Fig. 1 applied gate by gate, and phi(s) = <s|psi> (Methods A).
 * A projector |v><v| can be inserted on a wire; this is the value of one
 * sliced sub-network in the slicing identity of Methods C (TN equals the sum
 * over all fixed edge values), and a prefix of slices with D fixed wires is
 * one state-vector run with D projectors.
 *
 * Conventions: basis index i = sum_q bit_q(i) 2^q (qubit 0 least
 * significant); a two-qubit matrix is indexed by 2*bit(q0) + bit(q1).  Wire
 * (q, j) is the point on qubit q immediately before its j-th two-qubit gate
 * (0-based), after the single-qubit gates that precede that gate.
 *
 * Deliberately plain: one pass over the state per gate, no gate fusion, no
 * blocking.  Built with -ffp-contract=off.  Shares no code with the library.
 */
#include <complex.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

void sv_zero_state(cplx *psi, int n) {
  int64_t N = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; ++i) psi[i] = 0.0;
  psi[0] = 1.0;
}

/* psi <- (I x .. x g_q x .. x I) psi */
void sv_apply_1q(cplx *psi, int n, int q, const cplx *g) {
  int64_t N = (int64_t)1 << n;
  int64_t bq = (int64_t)1 << q;
  cplx g00 = g[0], g01 = g[1], g10 = g[2], g11 = g[3];
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; ++i) {
    if (i & bq) continue;
    cplx a0 = psi[i], a1 = psi[i | bq];
    psi[i] = g00 * a0 + g01 * a1;
    psi[i | bq] = g10 * a0 + g11 * a1;
  }
}

/* psi <- G_{q0 q1} psi with G indexed by 2*bit(q0) + bit(q1). */
void sv_apply_2q(cplx *psi, int n, int q0, int q1, const cplx *g) {
  int64_t N = (int64_t)1 << n;
  int64_t b0 = (int64_t)1 << q0, b1 = (int64_t)1 << q1;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; ++i) {
    if ((i & b0) || (i & b1)) continue;
    int64_t idx[4] = {i, i | b1, i | b0, i | b0 | b1};
    cplx a[4], r[4];
    for (int c = 0; c < 4; ++c) a[c] = psi[idx[c]];
    for (int rr = 0; rr < 4; ++rr) {
      cplx s = 0.0;
      for (int c = 0; c < 4; ++c) s += g[rr * 4 + c] * a[c];
      r[rr] = s;
    }
    for (int c = 0; c < 4; ++c) psi[idx[c]] = r[c];
  }
}

/* psi <- |v><v|_q psi */
void sv_project(cplx *psi, int n, int q, int v) {
  int64_t N = (int64_t)1 << n;
  int64_t bq = (int64_t)1 << q;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; ++i) {
    int bit = (i & bq) ? 1 : 0;
    if (bit != v) psi[i] = 0.0;
  }
}

/*
 * Run a circuit.  Gate g acts on nq[g] qubits q[2g], q[2g+1] with the
 * row-major matrix mat[16g ...].  Projectors: proj_q[p], proj_j[p],
 * proj_v[p] insert |v><v| on wire (q, j).  If stop_after_gate >= 0 the run
 * stops after that many gates (used by the per-layer norm check).
 */
int sv_run_circuit(cplx *psi, int n, int n_gates, const int32_t *nq,
                   const int32_t *q, const cplx *mat, int n_proj,
                   const int32_t *proj_q, const int32_t *proj_j,
                   const int32_t *proj_v, int stop_after_gate) {
  int *count2q = (int *)calloc((size_t)n, sizeof(int));
  if (!count2q) return -1;
  sv_zero_state(psi, n);
  int limit = stop_after_gate >= 0 ? stop_after_gate : n_gates;
  for (int g = 0; g < limit; ++g) {
    if (nq[g] == 1) {
      sv_apply_1q(psi, n, q[2 * g], mat + 16 * (int64_t)g);
    } else if (nq[g] == 2) {
      int qa = q[2 * g], qb = q[2 * g + 1];
      for (int p = 0; p < n_proj; ++p) {
        if ((proj_q[p] == qa && proj_j[p] == count2q[qa]) ||
            (proj_q[p] == qb && proj_j[p] == count2q[qb]))
          sv_project(psi, n, proj_q[p], proj_v[p]);
      }
      sv_apply_2q(psi, n, qa, qb, mat + 16 * (int64_t)g);
      count2q[qa]++;
      count2q[qb]++;
    } else {
      free(count2q);
      return -2;
    }
  }
  free(count2q);
  return 0;
}

void sv_gather(const cplx *psi, int64_t m, const uint64_t *idx, cplx *out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) out[i] = psi[idx[i]];
}

/* sum_i |psi_i|^2 */
double sv_norm2(const cplx *psi, int n) {
  int64_t N = (int64_t)1 << n;
  double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static)
  for (int64_t i = 0; i < N; ++i) {
    double re = creal(psi[i]), im = cimag(psi[i]);
    s += re * re + im * im;
  }
  return s;
}

/* Moments sum_i q_i^2 and sum_i q_i^3 of q_i = |psi_i|^2. */
void sv_moments(const cplx *psi, int n, double *m2, double *m3) {
  int64_t N = (int64_t)1 << n;
  double s2 = 0.0, s3 = 0.0;
#pragma omp parallel for reduction(+ : s2, s3) schedule(static)
  for (int64_t i = 0; i < N; ++i) {
    double re = creal(psi[i]), im = cimag(psi[i]);
    double p = re * re + im * im;
    s2 += p * p;
    s3 += p * p * p;
  }
  *m2 = s2;
  *m3 = s3;
}

/*
 * Exact sampling by inversion: u[] sorted ascending in [0, total); one
 * streaming pass over the cumulative distribution.
 */
void sv_sample_sorted(const cplx *psi, int n, int64_t m, const double *u_sorted,
                      uint64_t *out) {
  int64_t N = (int64_t)1 << n;
  double c = 0.0;
  int64_t j = 0;
  for (int64_t i = 0; i < N && j < m; ++i) {
    double re = creal(psi[i]), im = cimag(psi[i]);
    c += re * re + im * im;
    while (j < m && u_sorted[j] < c) out[j++] = (uint64_t)i;
  }
  while (j < m) out[j++] = (uint64_t)(N - 1);
}

/* Probabilities p_i = |psi_i|^2 written to a double array. */
void sv_probs(const cplx *psi, int n, double *p) {
  int64_t N = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; ++i) {
    double re = creal(psi[i]), im = cimag(psi[i]);
    p[i] = re * re + im * im;
  }
}
