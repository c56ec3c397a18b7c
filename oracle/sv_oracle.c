/*
 * Plain CPU oracle for the fused-operator state-vector path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file; only the tests, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code, header or table with the HIP
 * path.
 *
 * Conventions (Section II, "State and layout notation" and "Fused gates and
 * requests"):
 *   - a state of n qubits is 2^n complex128 amplitudes, stored interleaved
 *     (re, im) as doubles; basis index bit q holds qubit q, bit 0 least
 *     significant;
 *   - a k-qubit gate is a dense 2^k x 2^k complex matrix G, row-major and
 *     interleaved, with ordered targets (q_0..q_{k-1}); q_j supplies bit j of
 *     the row and column index.
 *
 * Every routine is the plain definition written out, with no blocking, fusion
 * or reordering.  OpenMP parallelises over independent amplitude groups only.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void orc_set_threads(int t) {
#ifdef _OPENMP
  if (t > 0) omp_set_num_threads(t);
#else
  (void)t;
#endif
}

/* Initialise |0...0>. */
void orc_zero_state(double *psi, int n) {
  int64_t dim = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
  for (int64_t x = 0; x < dim; ++x) {
    psi[2 * x] = 0.0;
    psi[2 * x + 1] = 0.0;
  }
  psi[0] = 1.0;
}

/*
 * Apply one gate (Section IV-B semantics; target j of the tuple is bit j of
 * G's row and column index, Section II).  Each group is the 2^k amplitudes
 * whose n-k non-target bits agree; the group is read, multiplied by G and
 * written back in place.
 *
 * For every x whose target bits are all zero, amplitude r of the group is
 * psi[x + sum_j ((r >> j) & 1) << q_j], and the new value of amplitude r is
 * sum_c G[r][c] * old amplitude c.
 */
int orc_apply_gate(double *psi, int n, const double *G, const int32_t *targets, int k) {
  if (k < 1 || k > n || k > 12) return -1;
  for (int j = 0; j < k; ++j) {
    if (targets[j] < 0 || targets[j] >= n) return -1;
    for (int i = 0; i < j; ++i)
      if (targets[i] == targets[j]) return -1;
  }
  const int64_t dim = (int64_t)1 << k;
  /* target positions in ascending order, for inserting zero bits */
  int sorted[16];
  for (int j = 0; j < k; ++j) sorted[j] = targets[j];
  for (int a = 1; a < k; ++a)
    for (int b = a; b > 0 && sorted[b - 1] > sorted[b]; --b) {
      int t = sorted[b];
      sorted[b] = sorted[b - 1];
      sorted[b - 1] = t;
    }
  int64_t *off = (int64_t *)malloc(sizeof(int64_t) * dim);
  for (int64_t r = 0; r < dim; ++r) {
    int64_t o = 0;
    for (int j = 0; j < k; ++j)
      if ((r >> j) & 1) o |= (int64_t)1 << targets[j];
    off[r] = o;
  }
  const int64_t ngroups = (int64_t)1 << (n - k);
#pragma omp parallel
  {
    double *a = (double *)malloc(sizeof(double) * 2 * dim);
    double *b = (double *)malloc(sizeof(double) * 2 * dim);
#pragma omp for schedule(static)
    for (int64_t g = 0; g < ngroups; ++g) {
      int64_t x = g;
      for (int j = 0; j < k; ++j) {
        int p = sorted[j];
        int64_t low = x & (((int64_t)1 << p) - 1);
        x = ((x >> p) << (p + 1)) | low;
      }
      for (int64_t c = 0; c < dim; ++c) {
        a[2 * c] = psi[2 * (x + off[c])];
        a[2 * c + 1] = psi[2 * (x + off[c]) + 1];
      }
      for (int64_t r = 0; r < dim; ++r) {
        double re = 0.0, im = 0.0;
        const double *row = G + 2 * r * dim;
        for (int64_t c = 0; c < dim; ++c) {
          double gr = row[2 * c], gi = row[2 * c + 1];
          re += gr * a[2 * c] - gi * a[2 * c + 1];
          im += gr * a[2 * c + 1] + gi * a[2 * c];
        }
        b[2 * r] = re;
        b[2 * r + 1] = im;
      }
      for (int64_t r = 0; r < dim; ++r) {
        psi[2 * (x + off[r])] = b[2 * r];
        psi[2 * (x + off[r]) + 1] = b[2 * r + 1];
      }
    }
    free(a);
    free(b);
  }
  free(off);
  return 0;
}

/* Apply a packed gate list in order (ks[i] targets each, matrices back to back). */
int orc_apply_circuit(double *psi, int n, int ngates, const int32_t *ks, const int32_t *targets,
                      const double *mats) {
  int64_t toff = 0, moff = 0;
  for (int i = 0; i < ngates; ++i) {
    int k = ks[i];
    int rc = orc_apply_gate(psi, n, mats + moff, targets + toff, k);
    if (rc) return rc;
    toff += k;
    moff += 2 * ((int64_t)1 << (2 * k));
  }
  return 0;
}

/* p_x = |psi_x|^2 in FP64. */
void orc_probs(const double *psi, int n, double *p) {
  int64_t dim = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
  for (int64_t x = 0; x < dim; ++x) p[x] = psi[2 * x] * psi[2 * x] + psi[2 * x + 1] * psi[2 * x + 1];
}

/*
 * Decode a physically stored state through a layout map (Section IV-D: the
 * physical index y has y_{L(q)} = x_q for logical index x).  out[x] = in[y].
 */
void orc_decode(const double *phys, int n, const int32_t *layout, double *logical) {
  int64_t dim = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
  for (int64_t x = 0; x < dim; ++x) {
    int64_t y = 0;
    for (int q = 0; q < n; ++q)
      if ((x >> q) & 1) y |= (int64_t)1 << layout[q];
    logical[2 * x] = phys[2 * y];
    logical[2 * x + 1] = phys[2 * y + 1];
  }
}

/* <Z_q> = sum_x |psi_x|^2 (1 - 2 x_q). */
double orc_expect_z(const double *psi, int n, int q) {
  int64_t dim = (int64_t)1 << n;
  double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static)
  for (int64_t x = 0; x < dim; ++x) {
    double p = psi[2 * x] * psi[2 * x] + psi[2 * x + 1] * psi[2 * x + 1];
    s += ((x >> q) & 1) ? -p : p;
  }
  return s;
}

/*
 * Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11):
 * ten rounds of two 32x32->64 multiplies with the published multipliers,
 * the key advanced by the published Weyl increments between rounds.
 */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0;
    c1 = n1;
    c2 = n2;
    c3 = n3;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

/* The 64-bit draw for shot s: key = seed, counter = (s, 0). */
uint64_t orc_shot_bits(uint64_t seed, uint64_t shot) {
  uint32_t ctr[4] = {(uint32_t)shot, (uint32_t)(shot >> 32), 0u, 0u};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t o[4];
  orc_philox4x32_10(ctr, key, o);
  return (uint64_t)o[0] | ((uint64_t)o[1] << 32);
}

/*
 * Inverse-CDF sampling with a strict upper bound (Section IV-E, "Sampling":
 * a zero-probability bin can never be selected).  Probabilities are taken to
 * fixed point, q_x = floor(p_x * 2^62), so that the cumulative sums are exact
 * integers; C(x) = sum_{y<=x} q_y, T = C(2^n - 1).  For shot s the 64-bit
 * draw r gives t = floor(r * T / 2^64) < T and the outcome is the smallest x
 * with C(x) > t.  This is the plain single-level CDF; no blocks.
 * Returns 0, or -1 when T == 0.
 */
int orc_sample(const double *p, int n, uint64_t seed, int64_t shots, uint64_t *out) {
  int64_t dim = (int64_t)1 << n;
  uint64_t *cdf = (uint64_t *)malloc(sizeof(uint64_t) * dim);
  if (!cdf) return -2;
  uint64_t acc = 0;
  for (int64_t x = 0; x < dim; ++x) {
    uint64_t q = (uint64_t)(p[x] * 0x1p62);
    acc += q;
    cdf[x] = acc;
  }
  uint64_t total = acc;
  if (total == 0) {
    free(cdf);
    return -1;
  }
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < shots; ++s) {
    uint64_t r = orc_shot_bits(seed, (uint64_t)s);
    uint64_t t = (uint64_t)(((unsigned __int128)r * total) >> 64);
    int64_t lo = 0, hi = dim - 1; /* smallest x with cdf[x] > t; cdf[dim-1] = total > t */
    while (lo < hi) {
      int64_t mid = lo + (hi - lo) / 2;
      if (cdf[mid] > t)
        hi = mid;
      else
        lo = mid + 1;
    }
    out[s] = (uint64_t)lo;
  }
  free(cdf);
  return 0;
}
