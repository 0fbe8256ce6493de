/*
 * The oracle: a plain, sequential FP64 dual-regularised tree Riccati recursion.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the CPU-baseline
 * leg of the benchmark may load this library.  It shares no code, header,
 * helper or table with the GPU solver.
 *
 * What it computes is the unique KKT solution of eq. (kkt) (Prop. 1) together
 * with the Riccati coefficients P_i (Thm. 1) and the feedback gains K_e
 * (eq. (factor-local)), by the standard sequential recursion that follows the
 * tree height (Sec. XI-A, the "CPU seq." baseline):
 *
 *   backward, children before parents (Lemma 5 and its proof):
 *     P_i = Q_i,  p_i = q_i
 *     for every child edge e = (i, j):
 *       F_j = I + Delta_j P_j,  W_j = P_j F_j^{-1}                 eq. (FW)
 *       f_j = Delta_j p_j - c_j,  g_j = p_j - W_j f_j              eq. (local-affine-solve)
 *       G_e = R_e + B_e^T W_j B_e,  H_e = B_e^T W_j A_e + M_e^T    eq. (factor-local)
 *       K_e = -G_e^{-1} H_e,  k_e = -G_e^{-1} (r_e + B_e^T g_j)
 *       A^cl_e = A_e + B_e K_e
 *       P_i += M_e K_e + A_e^T W_j A^cl_e                          proof of Lemma 5
 *       p_i += K_e^T r_e + (A^cl_e)^T g_j                          eq. (affine-message), d_e
 *   root:  x_rho = -F_rho^{-1} f_rho                               eq. (xroot)
 *   forward, parents before children (proof of Lemma 5):
 *     u_e = K_e x_i + k_e,  x_j = F_j^{-1} (A_e x_i + B_e u_e - f_j)
 *     y_i = P_i x_i + p_i                                          eq. (recover)
 *
 * Layout: row-major float64; node arrays indexed by node id, edge arrays by
 * the child id j of edge (parent[j], j) ("edge slot j"); the root's edge slot
 * of K and u is written as zero.  S is the paper's cross term M_e (n x m).
 * Small dense systems use the oracle's own LU with partial pivoting and
 * Cholesky below.  No recursion: the caterpillar trees are ~10^5 deep.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_BAD_TREE -1
#define OR_BAD_DIMS -2
#define OR_NOMEM -3
#define OR_SINGULAR -4
#define OR_NOT_PD -5

/* ----------------------------------------------------------- dense helpers */
/* C (r x c) = A (r x k) * B (k x c), with optional transposes of A, B as stored. */
static void mat_mul(int r, int k, int c, const double *A, int ta, const double *B, int tb,
                    double *C) {
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < c; ++j) {
      double s = 0.0;
      for (int l = 0; l < k; ++l) {
        double a = ta ? A[l * r + i] : A[i * k + l];
        double b = tb ? B[j * k + l] : B[l * c + j];
        s += a * b;
      }
      C[i * c + j] = s;
    }
}

/* y (r) = A (r x k) x (k), or A^T x when ta (A stored k x r). */
static void mat_vec(int r, int k, const double *A, int ta, const double *x, double *y) {
  for (int i = 0; i < r; ++i) {
    double s = 0.0;
    for (int l = 0; l < k; ++l) s += (ta ? A[l * r + i] : A[i * k + l]) * x[l];
    y[i] = s;
  }
}

/* In-place LU with partial pivoting of the d x d matrix M; piv receives the row order. */
static int lu_factor(int d, double *M, int *piv) {
  for (int i = 0; i < d; ++i) piv[i] = i;
  for (int k = 0; k < d; ++k) {
    int p = k;
    double best = fabs(M[k * d + k]);
    for (int i = k + 1; i < d; ++i)
      if (fabs(M[i * d + k]) > best) { best = fabs(M[i * d + k]); p = i; }
    if (best == 0.0) return OR_SINGULAR;
    if (p != k) {
      for (int j = 0; j < d; ++j) { double t = M[k * d + j]; M[k * d + j] = M[p * d + j]; M[p * d + j] = t; }
      int t = piv[k]; piv[k] = piv[p]; piv[p] = t;
    }
    for (int i = k + 1; i < d; ++i) {
      double l = M[i * d + k] / M[k * d + k];
      M[i * d + k] = l;
      for (int j = k + 1; j < d; ++j) M[i * d + j] -= l * M[k * d + j];
    }
  }
  return OR_OK;
}

/* Solve (LU) X = Bm for nr right-hand sides stored as the columns of Bm (d x nr). */
static void lu_solve(int d, const double *LU, const int *piv, int nr, double *Bm, double *tmp) {
  for (int c = 0; c < nr; ++c) {
    for (int i = 0; i < d; ++i) tmp[i] = Bm[piv[i] * nr + c];
    for (int i = 0; i < d; ++i)
      for (int j = 0; j < i; ++j) tmp[i] -= LU[i * d + j] * tmp[j];
    for (int i = d - 1; i >= 0; --i) {
      for (int j = i + 1; j < d; ++j) tmp[i] -= LU[i * d + j] * tmp[j];
      tmp[i] /= LU[i * d + i];
    }
    for (int i = 0; i < d; ++i) Bm[i * nr + c] = tmp[i];
  }
}

/* Lower Cholesky factor of the SPD d x d matrix M, in place (upper part unused). */
static int chol_factor(int d, double *M) {
  for (int j = 0; j < d; ++j) {
    double s = M[j * d + j];
    for (int k = 0; k < j; ++k) s -= M[j * d + k] * M[j * d + k];
    if (!(s > 0.0)) return OR_NOT_PD;
    double l = sqrt(s);
    M[j * d + j] = l;
    for (int i = j + 1; i < d; ++i) {
      double t = M[i * d + j];
      for (int k = 0; k < j; ++k) t -= M[i * d + k] * M[j * d + k];
      M[i * d + j] = t / l;
    }
  }
  return OR_OK;
}

/* Solve (L L^T) X = Bm, Bm d x nr. */
static void chol_solve(int d, const double *L, int nr, double *Bm) {
  for (int c = 0; c < nr; ++c) {
    for (int i = 0; i < d; ++i) {
      double t = Bm[i * nr + c];
      for (int k = 0; k < i; ++k) t -= L[i * d + k] * Bm[k * nr + c];
      Bm[i * nr + c] = t / L[i * d + i];
    }
    for (int i = d - 1; i >= 0; --i) {
      double t = Bm[i * nr + c];
      for (int k = i + 1; k < d; ++k) t -= L[k * d + i] * Bm[k * nr + c];
      Bm[i * nr + c] = t / L[i * d + i];
    }
  }
}

/* ----------------------------------------------------------- tree helpers */
/* Breadth-first order from the unique root; children visited in ascending id. */
static int bfs(int64_t N, const int64_t *parent, int64_t *order, int64_t *cstart, int64_t *kids) {
  int64_t root = -1;
  for (int64_t i = 0; i < N; ++i) {
    if (parent[i] < 0) {
      if (parent[i] != -1 || root >= 0) return OR_BAD_TREE;
      root = i;
    } else if (parent[i] >= N || parent[i] == i) {
      return OR_BAD_TREE;
    }
  }
  if (root < 0) return OR_BAD_TREE;
  memset(cstart, 0, sizeof(int64_t) * (size_t)(N + 1));
  for (int64_t i = 0; i < N; ++i)
    if (parent[i] >= 0) cstart[parent[i] + 1]++;
  for (int64_t i = 0; i < N; ++i) cstart[i + 1] += cstart[i];
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
  if (!fill) return OR_NOMEM;
  for (int64_t i = 0; i < N; ++i) fill[i] = cstart[i];
  for (int64_t i = 0; i < N; ++i)
    if (parent[i] >= 0) kids[fill[parent[i]]++] = i;
  free(fill);
  int64_t head = 0, tail = 0;
  order[tail++] = root;
  while (head < tail) {
    int64_t v = order[head++];
    for (int64_t c = cstart[v]; c < cstart[v + 1]; ++c) order[tail++] = kids[c];
  }
  return tail == N ? OR_OK : OR_BAD_TREE; /* a cycle leaves nodes unreached */
}

/* ----------------------------------------------------------- the recursion */
int oracle_tree_riccati(int64_t N, int32_t n, int32_t m, const int64_t *parent,
                        const double *Q, const double *q, const double *c, const double *Delta,
                        const double *R, const double *S, const double *r, const double *A,
                        const double *B, double *K, double *P, double *x, double *u, double *lam,
                        double *p_out, double *kff_out) {
  if (N < 1) return OR_BAD_TREE;
  if (n < 1 || m < 1 || n > 64 || m > 64) return OR_BAD_DIMS;
  const size_t nn = (size_t)n * n, nm = (size_t)n * m, mm = (size_t)m * m;
  int64_t *order = malloc(sizeof(int64_t) * (size_t)N);
  int64_t *cstart = malloc(sizeof(int64_t) * (size_t)(N + 1));
  int64_t *kids = malloc(sizeof(int64_t) * (size_t)N);
  double *p = malloc(sizeof(double) * (size_t)N * n);
  double *f = malloc(sizeof(double) * (size_t)N * n);
  double *kff = malloc(sizeof(double) * (size_t)N * m);
  double *work = malloc(sizeof(double) * (8 * nn + 4 * nm + 4 * mm + 8 * (size_t)(n + m)));
  int *piv = malloc(sizeof(int) * (size_t)(n + m));
  int rc = OR_OK;
  if (!order || !cstart || !kids || !p || !f || !kff || !work || !piv) { rc = OR_NOMEM; goto done; }
  rc = bfs(N, parent, order, cstart, kids);
  if (rc) goto done;

  double *F = work, *W = F + nn, *T1 = W + nn, *T2 = T1 + nn, *Acl = T2 + nn;
  double *BtW = Acl + nn;            /* m x n */
  double *G = BtW + nm;              /* m x m */
  double *H = G + mm;                /* m x n */
  double *gv = H + nm;               /* n */
  double *kv = gv + n;               /* m */
  double *tv = kv + m;               /* n + m scratch */
  double *tv2 = tv + (n + m);        /* n + m scratch */

  /* backward pass: reverse BFS order visits every child before its parent */
  for (int64_t t = N - 1; t >= 0; --t) {
    int64_t i = order[t];
    double *Pi = P + (size_t)i * nn, *pi = p + (size_t)i * n;
    memcpy(Pi, Q + (size_t)i * nn, sizeof(double) * nn);
    memcpy(pi, q + (size_t)i * n, sizeof(double) * n);
    for (int64_t cc = cstart[i]; cc < cstart[i + 1]; ++cc) {
      int64_t j = kids[cc];
      const double *Pj = P + (size_t)j * nn, *pj = p + (size_t)j * n;
      const double *Dj = Delta + (size_t)j * nn;
      const double *Ae = A + (size_t)j * nn, *Be = B + (size_t)j * nm;
      const double *Re = R + (size_t)j * mm, *Se = S + (size_t)j * nm, *re = r + (size_t)j * m;
      /* F_j = I + Delta_j P_j */
      mat_mul(n, n, n, Dj, 0, Pj, 0, F);
      for (int a = 0; a < n; ++a) F[a * n + a] += 1.0;
      /* W_j = P_j F_j^{-1}: W F = P, i.e. F^T W^T = P^T; solve for W^T then transpose */
      for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) T1[a * n + b] = F[b * n + a]; /* F^T */
      for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) T2[a * n + b] = Pj[b * n + a]; /* P^T */
      if ((rc = lu_factor(n, T1, piv))) goto done;
      lu_solve(n, T1, piv, n, T2, tv);
      for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) W[a * n + b] = T2[b * n + a];
      /* f_j = Delta_j p_j - c_j ; g_j = p_j - W_j f_j */
      double *fj = f + (size_t)j * n;
      mat_vec(n, n, Dj, 0, pj, fj);
      for (int a = 0; a < n; ++a) fj[a] -= c[(size_t)j * n + a];
      mat_vec(n, n, W, 0, fj, tv);
      for (int a = 0; a < n; ++a) gv[a] = pj[a] - tv[a];
      /* G = R + B^T W B ; H = B^T W A + S^T */
      mat_mul(m, n, n, Be, 1, W, 0, BtW);
      mat_mul(m, n, m, BtW, 0, Be, 0, G);
      for (size_t a = 0; a < mm; ++a) G[a] += Re[a];
      mat_mul(m, n, n, BtW, 0, Ae, 0, H);
      for (int a = 0; a < m; ++a)
        for (int b = 0; b < n; ++b) H[a * n + b] += Se[b * m + a];
      /* K = -G^{-1} H ; k = -G^{-1}(r + B^T g) */
      double *Ke = K + (size_t)j * nm;
      if ((rc = chol_factor(m, G))) goto done;
      memcpy(Ke, H, sizeof(double) * nm);
      chol_solve(m, G, n, Ke);
      for (size_t a = 0; a < nm; ++a) Ke[a] = -Ke[a];
      mat_vec(m, n, Be, 1, gv, kv);
      for (int a = 0; a < m; ++a) kv[a] = -(kv[a] + re[a]);
      chol_solve(m, G, 1, kv);
      memcpy(kff + (size_t)j * m, kv, sizeof(double) * m);
      /* A^cl = A + B K */
      mat_mul(n, m, n, Be, 0, Ke, 0, Acl);
      for (size_t a = 0; a < nn; ++a) Acl[a] += Ae[a];
      /* P_i += M_e K_e + A_e^T W_j A^cl_e */
      mat_mul(n, m, n, Se, 0, Ke, 0, T1);
      mat_mul(n, n, n, W, 0, Acl, 0, T2);
      for (size_t a = 0; a < nn; ++a) Pi[a] += T1[a];
      mat_mul(n, n, n, Ae, 1, T2, 0, T1);
      for (size_t a = 0; a < nn; ++a) Pi[a] += T1[a];
      /* p_i += K_e^T r_e + (A^cl_e)^T g_j */
      mat_vec(n, m, Ke, 1, re, tv);
      mat_vec(n, n, Acl, 1, gv, tv2);
      for (int a = 0; a < n; ++a) pi[a] += tv[a] + tv2[a];
    }
  }

  /* root: F x = -f */
  {
    int64_t rt = order[0];
    const double *Pr = P + (size_t)rt * nn, *pr = p + (size_t)rt * n, *Dr = Delta + (size_t)rt * nn;
    double *fr = f + (size_t)rt * n;
    mat_mul(n, n, n, Dr, 0, Pr, 0, F);
    for (int a = 0; a < n; ++a) F[a * n + a] += 1.0;
    mat_vec(n, n, Dr, 0, pr, fr);
    for (int a = 0; a < n; ++a) fr[a] -= c[(size_t)rt * n + a];
    if ((rc = lu_factor(n, F, piv))) goto done;
    double *xr = x + (size_t)rt * n;
    for (int a = 0; a < n; ++a) xr[a] = -fr[a];
    lu_solve(n, F, piv, 1, xr, tv);
    memset(K + (size_t)rt * nm, 0, sizeof(double) * nm);
    memset(u + (size_t)rt * m, 0, sizeof(double) * m);
    memset(kff + (size_t)rt * m, 0, sizeof(double) * m);
  }

  /* forward pass in BFS order */
  for (int64_t t = 1; t < N; ++t) {
    int64_t j = order[t], i = parent[j];
    const double *xi = x + (size_t)i * n;
    const double *Ke = K + (size_t)j * nm, *Ae = A + (size_t)j * nn, *Be = B + (size_t)j * nm;
    const double *Pj = P + (size_t)j * nn, *Dj = Delta + (size_t)j * nn;
    double *ue = u + (size_t)j * m, *xj = x + (size_t)j * n;
    mat_vec(m, n, Ke, 0, xi, ue);
    for (int a = 0; a < m; ++a) ue[a] += kff[(size_t)j * m + a];
    mat_vec(n, n, Ae, 0, xi, tv);
    mat_vec(n, m, Be, 0, ue, tv2);
    for (int a = 0; a < n; ++a) xj[a] = tv[a] + tv2[a] - f[(size_t)j * n + a];
    mat_mul(n, n, n, Dj, 0, Pj, 0, F);
    for (int a = 0; a < n; ++a) F[a * n + a] += 1.0;
    if ((rc = lu_factor(n, F, piv))) goto done;
    lu_solve(n, F, piv, 1, xj, tv);
  }
  for (int64_t i = 0; i < N; ++i) {
    mat_vec(n, n, P + (size_t)i * nn, 0, x + (size_t)i * n, lam + (size_t)i * n);
    for (int a = 0; a < n; ++a) lam[(size_t)i * n + a] += p[(size_t)i * n + a];
  }
  if (p_out) memcpy(p_out, p, sizeof(double) * (size_t)N * n);
  if (kff_out) memcpy(kff_out, kff, sizeof(double) * (size_t)N * m);

done:
  free(order); free(cstart); free(kids); free(p); free(f); free(kff); free(work); free(piv);
  return rc;
}

/* Batch entry for the multi-core CPU baseline: trees are independent, so each
 * of nthreads POSIX threads runs the plain recursion above on its own trees. */
#include <pthread.h>
typedef struct {
  int64_t count;
  const int64_t *Ns;
  int32_t n, m;
  const int64_t *const *parents;
  const double *const *data; /* 9 arrays per tree: Q q c Delta R S r A B */
  double *const *out;        /* 5 arrays per tree: K P x u lam */
  int64_t next;
  pthread_mutex_t mu;
  int rc;
} batch_job;

static void *batch_worker(void *arg) {
  batch_job *jb = (batch_job *)arg;
  for (;;) {
    pthread_mutex_lock(&jb->mu);
    int64_t t = jb->next++;
    pthread_mutex_unlock(&jb->mu);
    if (t >= jb->count) break;
    const double *const *d = jb->data + 9 * t;
    double *const *o = jb->out + 5 * t;
    int rc = oracle_tree_riccati(jb->Ns[t], jb->n, jb->m, jb->parents[t], d[0], d[1], d[2], d[3],
                                 d[4], d[5], d[6], d[7], d[8], o[0], o[1], o[2], o[3], o[4], NULL,
                                 NULL);
    if (rc) {
      pthread_mutex_lock(&jb->mu);
      jb->rc = rc;
      pthread_mutex_unlock(&jb->mu);
    }
  }
  return NULL;
}

int oracle_tree_riccati_batch(int64_t count, const int64_t *Ns, int32_t n, int32_t m,
                              const int64_t *const *parents, const double *const *data,
                              double *const *out, int32_t nthreads) {
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  batch_job jb = {count, Ns, n, m, parents, data, out, 0, PTHREAD_MUTEX_INITIALIZER, OR_OK};
  pthread_t th[256];
  for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, batch_worker, &jb);
  for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
  return jb.rc;
}
