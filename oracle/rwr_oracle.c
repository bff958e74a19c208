/*
 * Oracle for random walk with restart (RWR) on dynamic graphs -- TEST
 * INFRASTRUCTURE ONLY.  Plain, single-threaded, FP64 C.  Only the tests, the
 * smoke check and the benchmark's CPU-baseline leg load this file's library;
 * the product path never does, and this file shares no code with it.
 *
 * Graphs are plain directed edge lists (src[e], dst[e]); the row-normalised
 * adjacency of Section 2.1 (and its symbol table) is A~[u][v] = 1/d_out(u) for
 * every edge (u, v), with rows of dead ends (d_out = 0) all zero.
 *
 * Functions
 *   orc_cpi   cumulative power iteration of Section 2.2 for any seed vector
 *   orc_rwr   static RWR of Eq. (1): CPI from c*e_s, then the dead-end
 *             normalisation of Theorem 4 (Section 3.4.2)
 *   orc_osp   the offset-score-propagation update of Section 3.1 /
 *             Algorithm 1 (OSP, and OSP-T with a larger tolerance)
 *   orc_dead_end_reachable  breadth-first search used by orc_rwr
 *
 * Readings of the paper taken here (each is listed with its reason in the
 * design notes of the repository):
 *   - the accumulated offset r_offset includes x^(0) = q_offset, as the sums of
 *     Section 3.1 and the proof of Theorem 1 run from i = 0;
 *   - the loop of Algorithm 1 computes x^(i) first and then tests its L1 norm
 *     (at least one iteration always runs);
 *   - dead ends: scores are computed on the sub-stochastic matrix and scaled
 *     by the reciprocal of their L1 norm (Theorem 4).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ENOMEM -2
#define ORC_ENOCONV -6

/* Out-degree of every node: number of edges whose source it is. */
static int64_t *out_degrees(int64_t n, int64_t m, const int32_t *src) {
  int64_t *deg = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
  if (!deg) return NULL;
  for (int64_t e = 0; e < m; ++e) deg[src[e]] += 1;
  return deg;
}

static int check_edges(int64_t n, int64_t m, const int32_t *src, const int32_t *dst) {
  for (int64_t e = 0; e < m; ++e) {
    if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n) return ORC_EINVAL;
  }
  return ORC_OK;
}

/* y = (1-c) * A~^T x  for the graph (n, m, src, dst) with out-degrees deg.
 * (A~^T x)[v] = sum over edges (u, v) of x[u] / d_out(u). */
static void propagate(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, const int64_t *deg,
                      double c, const double *x, double *y) {
  for (int64_t v = 0; v < n; ++v) y[v] = 0.0;
  for (int64_t e = 0; e < m; ++e) {
    int32_t u = src[e];
    y[dst[e]] += x[u] / (double)deg[u];
  }
  for (int64_t v = 0; v < n; ++v) y[v] *= (1.0 - c);
}

static double l1(int64_t n, const double *x) {
  double s = 0.0;
  for (int64_t v = 0; v < n; ++v) s += fabs(x[v]);
  return s;
}

/*
 * Cumulative power iteration (Section 2.2):
 *   x^(0) = q,  x^(i) = (1-c) A~^T x^(i-1),  r = sum_{i>=0} x^(i),
 * summed until ||x^(i)||_1 <= tol (i >= 1).  `norms` (nullable, max_iter+1
 * entries) receives ||x^(i)||_1 for i = 0..iters.  Returns the number of
 * iterations in *iters, ORC_ENOCONV if max_iter is reached first.
 */
int orc_cpi(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, const double *q, double c, double tol,
            int32_t max_iter, double *r, double *norms, int32_t *iters) {
  if (n <= 0 || m < 0 || !(c > 0.0 && c < 1.0) || max_iter < 1) return ORC_EINVAL;
  if (check_edges(n, m, src, dst)) return ORC_EINVAL;
  int64_t *deg = out_degrees(n, m, src);
  double *x = (double *)malloc((size_t)n * sizeof(double));
  double *y = (double *)malloc((size_t)n * sizeof(double));
  if (!deg || !x || !y) {
    free(deg), free(x), free(y);
    return ORC_ENOMEM;
  }
  for (int64_t v = 0; v < n; ++v) x[v] = q[v], r[v] = q[v];
  if (norms) norms[0] = l1(n, x);
  int status = ORC_ENOCONV;
  int32_t i = 0;
  while (i < max_iter) {
    ++i;
    propagate(n, m, src, dst, deg, c, x, y);
    for (int64_t v = 0; v < n; ++v) r[v] += y[v];
    double nrm = l1(n, y);
    if (norms) norms[i] = nrm;
    double *t = x;
    x = y, y = t;
    if (nrm <= tol) {
      status = ORC_OK;
      break;
    }
  }
  *iters = i;
  free(deg), free(x), free(y);
  return status;
}

/* 1 if some node reachable from `seed` along out-edges has no out-edges. */
int orc_dead_end_reachable(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, int32_t seed) {
  if (seed < 0 || seed >= n) return 0;
  int64_t *deg = out_degrees(n, m, src);
  int64_t *start = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  int32_t *adj = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
  int32_t *queue = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  char *seen = (char *)calloc((size_t)n, 1);
  int found = 0;
  if (!deg || !start || !adj || !queue || !seen) {
    found = -1;
    goto done;
  }
  for (int64_t v = 0; v < n; ++v) start[v + 1] = start[v] + deg[v];
  {
    int64_t *fill = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!fill) {
      found = -1;
      goto done;
    }
    for (int64_t v = 0; v < n; ++v) fill[v] = start[v];
    for (int64_t e = 0; e < m; ++e) adj[fill[src[e]]++] = dst[e];
    free(fill);
  }
  int64_t head = 0, tail = 0;
  queue[tail++] = seed;
  seen[seed] = 1;
  while (head < tail) {
    int32_t u = queue[head++];
    if (deg[u] == 0) {
      found = 1;
      break;
    }
    for (int64_t k = start[u]; k < start[u + 1]; ++k) {
      int32_t v = adj[k];
      if (!seen[v]) seen[v] = 1, queue[tail++] = v;
    }
  }
done:
  free(deg), free(start), free(adj), free(queue), free(seen);
  return found;
}

/*
 * Static RWR of Eq. (1) for seed s: CPI (Section 2.2) from q_CPI = c * e_s to
 * tolerance `tol`; if a dead end is reachable from s the result is divided by
 * its L1 norm (Theorem 4).
 */
int orc_rwr(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, int32_t seed, double c, double tol,
            int32_t max_iter, double *r, int32_t *iters) {
  if (seed < 0 || seed >= n) return ORC_EINVAL;
  double *q = (double *)calloc((size_t)n, sizeof(double));
  if (!q) return ORC_ENOMEM;
  q[seed] = c;
  int st = orc_cpi(n, m, src, dst, q, c, tol, max_iter, r, NULL, iters);
  free(q);
  if (st != ORC_OK) return st;
  int de = orc_dead_end_reachable(n, m, src, dst, seed);
  if (de < 0) return ORC_ENOMEM;
  if (de) {
    double s = l1(n, r);
    for (int64_t v = 0; v < n; ++v) r[v] /= s;
  }
  return ORC_OK;
}

/*
 * One OSP / OSP-T update (Section 3.1, Algorithm 1; Section 3.2 for OSP-T).
 *   old graph (n_old, m_old, src_old, dst_old) with scores r_old[n_old];
 *   new graph (n_new >= n_old, ...): nodes n_old..n_new-1 are inserted nodes
 *   whose old rows, columns and scores are zero (Section 3.4.1).
 *
 *   q_offset = (1-c)(B~^T - A~^T) r_old
 *   x^(0) = q_offset, r_offset = x^(0)
 *   repeat: x^(i) = (1-c) B~^T x^(i-1); r_offset += x^(i)  until ||x^(i)||_1 <= eps
 *   r_new = r_old + r_offset
 *
 * renorm: 0 = Theorem 4 as the paper states it (divide by the L1 norm when a
 * dead end is reachable from `seed` in the new graph); 1 = divide by the
 * signed sum of r_new always; 2 = never.
 * Outputs: r_new[n_new], q_off[n_new] (nullable), norms[max_iter+1] (nullable,
 * ||x^(i)||_1 for i = 0..iters), *iters.
 */
int orc_osp(int64_t n_old, int64_t m_old, const int32_t *src_old, const int32_t *dst_old, int64_t n_new,
            int64_t m_new, const int32_t *src_new, const int32_t *dst_new, const double *r_old, double c,
            double eps, int32_t max_iter, int32_t renorm, int32_t seed, double *r_new, double *q_off,
            double *norms, int32_t *iters) {
  if (n_old <= 0 || n_new < n_old || !(c > 0.0 && c < 1.0) || max_iter < 1) return ORC_EINVAL;
  if (check_edges(n_old, m_old, src_old, dst_old) || check_edges(n_new, m_new, src_new, dst_new))
    return ORC_EINVAL;
  int64_t *deg_a = out_degrees(n_old, m_old, src_old);
  int64_t *deg_b = out_degrees(n_new, m_new, src_new);
  double *rold = (double *)calloc((size_t)n_new, sizeof(double));
  double *qa = (double *)malloc((size_t)n_new * sizeof(double));
  double *qb = (double *)malloc((size_t)n_new * sizeof(double));
  double *x = (double *)malloc((size_t)n_new * sizeof(double));
  double *y = (double *)malloc((size_t)n_new * sizeof(double));
  double *roff = (double *)malloc((size_t)n_new * sizeof(double));
  int status = ORC_ENOMEM;
  if (!deg_a || !deg_b || !rold || !qa || !qb || !x || !y || !roff) goto out;
  for (int64_t v = 0; v < n_old; ++v) rold[v] = r_old[v];

  /* q_offset = (1-c) B~^T r_old - (1-c) A~^T r_old */
  propagate(n_old, m_old, src_old, dst_old, deg_a, c, rold, qa);
  for (int64_t v = n_old; v < n_new; ++v) qa[v] = 0.0;
  propagate(n_new, m_new, src_new, dst_new, deg_b, c, rold, qb);
  for (int64_t v = 0; v < n_new; ++v) x[v] = qb[v] - qa[v];
  if (q_off)
    for (int64_t v = 0; v < n_new; ++v) q_off[v] = x[v];

  for (int64_t v = 0; v < n_new; ++v) roff[v] = x[v];
  if (norms) norms[0] = l1(n_new, x);
  status = ORC_ENOCONV;
  int32_t i = 0;
  while (i < max_iter) {
    ++i;
    propagate(n_new, m_new, src_new, dst_new, deg_b, c, x, y);
    for (int64_t v = 0; v < n_new; ++v) roff[v] += y[v];
    double nrm = l1(n_new, y);
    if (norms) norms[i] = nrm;
    double *t = x;
    x = y, y = t;
    if (nrm <= eps) {
      status = ORC_OK;
      break;
    }
  }
  *iters = i;
  for (int64_t v = 0; v < n_new; ++v) r_new[v] = rold[v] + roff[v];

  if (renorm == 0) {
    int de = orc_dead_end_reachable(n_new, m_new, src_new, dst_new, seed);
    if (de < 0) {
      status = ORC_ENOMEM;
      goto out;
    }
    if (de) {
      double s = l1(n_new, r_new);
      for (int64_t v = 0; v < n_new; ++v) r_new[v] /= s;
    }
  } else if (renorm == 1) {
    double s = 0.0;
    for (int64_t v = 0; v < n_new; ++v) s += r_new[v];
    for (int64_t v = 0; v < n_new; ++v) r_new[v] /= s;
  }
out:
  free(deg_a), free(deg_b), free(rold), free(qa), free(qb), free(x), free(y), free(roff);
  return status;
}
