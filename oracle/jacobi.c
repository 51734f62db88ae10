/*
 * Oracle (test infrastructure only; never part of the product path).
 *
 * Plain FP64 cyclic Jacobi eigensolver for a dense symmetric matrix, used to
 * form the exact prescribed-index reflector R_k = I - 2 Q_k Q_k^T of the
 * paper's eq. (Rk_intro) / eq. (Pk), which Prop. 2.1 (exact reflector
 * identity) equates with sgn(H - sI) for every s in (lambda_k, lambda_{k+1}).
 *
 * Method: classical two-sided Jacobi.  One sweep rotates every index pair
 * (p, q), p < q, exactly once.  Pairs are visited in the round-robin
 * ("tournament") order: a sweep is d-1 rounds of d/2 disjoint pairs (d even;
 * an odd d gets one dummy index that is skipped).  Rotations of disjoint
 * pairs commute and each one changes only its own 2x2 diagonal block, so
 * computing all angles of a round from the current matrix and applying them
 * together equals applying them one after the other; the round is therefore
 * applied as A <- J^T A J with J the product of the round's rotations, which
 * lets OpenMP split the work over rows and pairs.
 *
 * Rotation (Rutishauser's stable form): with theta = (a_qq - a_pp)/(2 a_pq),
 * t = sign(theta)/(|theta| + sqrt(theta^2 + 1)), c = 1/sqrt(1 + t^2), s = t c,
 * the updated block is a_pp - t a_pq, a_qq + t a_pq and a zero off-diagonal.
 * A rotation is skipped when a_pq is negligible next to both diagonal
 * entries (adding 100 |a_pq| leaves both unchanged in FP64); the iteration
 * stops after a sweep that applied no rotation, or after max_sweeps.
 *
 * Storage: A, V row-major d x d; V[i*d + j] is entry i of eigenvector j.
 * Eigenvalues are returned ascending with V's columns permuted alike.
 *
 * Nothing here is shared with the GPU library.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Round r of the round-robin schedule on m (even) players: player m-1 is
 * fixed, the others rotate.  Writes m/2 pairs (P[i], Q[i]). */
static void tournament_round(int64_t m, int64_t r, int64_t *P, int64_t *Q) {
  int64_t half = m / 2;
  for (int64_t i = 0; i < half; ++i) {
    int64_t a, b;
    if (i == 0) {
      a = m - 1;
      b = r % (m - 1);
    } else {
      a = (r + i) % (m - 1);
      b = (r + (m - 1) - i) % (m - 1);
    }
    P[i] = a < b ? a : b;
    Q[i] = a < b ? b : a;
  }
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads of the following solves (n >= 1); returns the number in force. */
int oracle_set_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

/* Returns the number of sweeps used, or -1 on bad arguments / no memory.
 * A is overwritten (its diagonal holds the unsorted eigenvalues on exit). */
int oracle_jacobi_eig(int64_t d, double *A, double *w, double *V,
                      int max_sweeps) {
  if (d < 1 || !A || !w || !V) return -1;
  int64_t m = (d % 2 == 0) ? d : d + 1; /* players incl. one dummy */
  int64_t half = m / 2;
  int64_t *P = (int64_t *)malloc(sizeof(int64_t) * half);
  int64_t *Q = (int64_t *)malloc(sizeof(int64_t) * half);
  double *C = (double *)malloc(sizeof(double) * half);
  double *S = (double *)malloc(sizeof(double) * half);
  double *T = (double *)malloc(sizeof(double) * half);
  double *App = (double *)malloc(sizeof(double) * half);
  double *Aqq = (double *)malloc(sizeof(double) * half);
  double *Apq = (double *)malloc(sizeof(double) * half);
  int *active = (int *)malloc(sizeof(int) * half);
  if (!P || !Q || !C || !S || !T || !App || !Aqq || !Apq || !active) {
    free(P); free(Q); free(C); free(S); free(T); free(App); free(Aqq); free(Apq); free(active);
    return -1;
  }
  for (int64_t i = 0; i < d; ++i)
    for (int64_t j = 0; j < d; ++j) V[i * d + j] = (i == j) ? 1.0 : 0.0;

  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    int64_t applied = 0;
    for (int64_t r = 0; r < m - 1; ++r) {
      tournament_round(m, r, P, Q);
      int64_t nact = 0;
      /* Angles of this round, all from the current matrix. */
      for (int64_t i = 0; i < half; ++i) {
        int64_t p = P[i], q = Q[i];
        active[i] = 0;
        if (q >= d) continue; /* dummy player */
        double apq = A[p * d + q];
        double app = A[p * d + p], aqq = A[q * d + q];
        double g = 100.0 * fabs(apq);
        if (apq == 0.0 || (fabs(app) + g == fabs(app) && fabs(aqq) + g == fabs(aqq))) {
          A[p * d + q] = 0.0;
          A[q * d + p] = 0.0;
          continue;
        }
        double theta = (aqq - app) / (2.0 * apq);
        double t;
        if (fabs(theta) > 1e150) {
          t = 0.5 / theta;
        } else {
          t = 1.0 / (fabs(theta) + sqrt(theta * theta + 1.0));
          if (theta < 0.0) t = -t;
        }
        double c = 1.0 / sqrt(1.0 + t * t);
        C[i] = c;
        S[i] = t * c;
        T[i] = t;
        App[i] = app;
        Aqq[i] = aqq;
        Apq[i] = apq;
        active[i] = 1;
        ++nact;
      }
      if (nact == 0) continue;
      applied += nact;
      /* Column part: A <- A J and V <- V J, row by row. */
#pragma omp parallel for schedule(static)
      for (int64_t row = 0; row < d; ++row) {
        double *a = A + row * d, *v = V + row * d;
        for (int64_t i = 0; i < half; ++i) {
          if (!active[i]) continue;
          int64_t p = P[i], q = Q[i];
          double c = C[i], s = S[i];
          double x = a[p], y = a[q];
          a[p] = c * x - s * y;
          a[q] = s * x + c * y;
          x = v[p];
          y = v[q];
          v[p] = c * x - s * y;
          v[q] = s * x + c * y;
        }
      }
      /* Row part: A <- J^T A, pair by pair (rows p and q). */
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < half; ++i) {
        if (!active[i]) continue;
        int64_t p = P[i], q = Q[i];
        double c = C[i], s = S[i];
        double *ap = A + p * d, *aq = A + q * d;
        for (int64_t col = 0; col < d; ++col) {
          double x = ap[col], y = aq[col];
          ap[col] = c * x - s * y;
          aq[col] = s * x + c * y;
        }
      }
      /* Rutishauser: the rotated 2x2 blocks take their closed form
       * (diagonal a_pp - t a_pq, a_qq + t a_pq; off-diagonal exactly 0). */
      for (int64_t i = 0; i < half; ++i) {
        if (!active[i]) continue;
        int64_t p = P[i], q = Q[i];
        A[p * d + p] = App[i] - T[i] * Apq[i];
        A[q * d + q] = Aqq[i] + T[i] * Apq[i];
        A[p * d + q] = 0.0;
        A[q * d + p] = 0.0;
      }
    }
    if (applied == 0) break;
  }

  /* Sort eigenvalues ascending (insertion order on an index array). */
  int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * d);
  double *tmp = (double *)malloc(sizeof(double) * d * d);
  if (!idx || !tmp) {
    free(idx); free(tmp);
    free(P); free(Q); free(C); free(S); free(T); free(App); free(Aqq); free(Apq); free(active);
    return -1;
  }
  for (int64_t i = 0; i < d; ++i) idx[i] = i;
  for (int64_t i = 1; i < d; ++i) {
    int64_t key = idx[i];
    double kv = A[key * d + key];
    int64_t j = i - 1;
    while (j >= 0 && A[idx[j] * d + idx[j]] > kv) {
      idx[j + 1] = idx[j];
      --j;
    }
    idx[j + 1] = key;
  }
  for (int64_t j = 0; j < d; ++j) w[j] = A[idx[j] * d + idx[j]];
  memcpy(tmp, V, sizeof(double) * d * d);
  for (int64_t i = 0; i < d; ++i)
    for (int64_t j = 0; j < d; ++j) V[i * d + j] = tmp[i * d + idx[j]];
  free(idx); free(tmp);
  free(P); free(Q); free(C); free(S); free(T); free(App); free(Aqq); free(Apq); free(active);
  return sweep;
}
