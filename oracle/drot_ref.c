/*
 * drot_ref.c -- plain, slow FP64 CPU oracle for DROT.
 *
 * TEST INFRASTRUCTURE ONLY.  The test-suite, the package's smoke check and the
 * benchmark's CPU-baseline leg are the only code that may load this library.
 * It shares no code, header or helper with the GPU implementation.
 *
 * What it follows (Mai, Lindbaeck, Johansson, "A Fast and Accurate Splitting
 * Method for Optimal Transport"):
 *   - Algorithm 1 (DROT), with the initial shifts of its first step, the a, b,
 *     alpha initialisation of its second step, the clamped X-update, the
 *     residuals r, s and beta, the two shift updates (which use the OLD a, b,
 *     alpha) and the three accumulator updates, in that order.
 *   - The stopping criteria of Section 3 ("Stopping criteria"): r_primal,
 *     r_dual and the duality gap, with the implicit dual variables
 *     mu = phi/rho and nu = varphi/rho (eq. dual:var in Appendix A).
 *
 * Notation: the paper's row shift is phi (length m) and its column shift is
 * varphi (length n); here the column shift is called psi.  X is stored
 * row-major with leading dimension n (row i is source i, column j target j).
 *
 * Readings of points the paper leaves open (each documented with the design):
 *   - Relative stopping test: eps_p = r_primal / sqrt(|p|^2 + |q|^2),
 *     eps_d = r_dual / |C|_F, eps_g = gap / max(|pobj|, |dobj|, 1e-300);
 *     stop when max(eps_p, eps_d, eps_g) <= tol (tol_mode 0), or when
 *     max(r_primal, r_dual, gap) <= tol (tol_mode 1).
 *   - r_dual is evaluated while C is read for the X-update, i.e. at the
 *     shifts that enter the update (one iteration behind r_primal and gap).
 *   - beta is taken from the row residual r (fT r / (m+n)).
 *   - Warm start: phi_0, psi_0 may be nonzero; then a_0 = Y_0 e - p and
 *     b_0 = Y_0^T f - q with Y_0 = X_0 + phi_0 e^T + f psi_0^T.
 * Compiled with -ffp-contract=off; every sum runs in a fixed order.
 *
 * Threads: built with -fopenmp (a second library, used only to time the
 * oracle on every core) the row loop of the sweep is split into T contiguous
 * row ranges, one per thread; each range keeps its own column sums and cost
 * and r_dual sums in row order, and the T partials are added in range order.
 * With one thread (the default build) this is exactly the row-major order of
 * a single loop.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define REF_OK 0
#define REF_MAXITER 1
#define REF_EINVAL -1
#define REF_ENOMEM -4

/* info[] slots written by drot_ref_solve / drot_ref_eval */
enum {
  I_ITERS = 0, I_STATUS, I_POBJ, I_DOBJ, I_RP, I_RD, I_GAP,
  I_EPS_P, I_EPS_D, I_EPS_G, I_ALPHA, I_NORMC, I_NORMPQ, I_NINFO
};

static double maxd(double a, double b) { return a > b ? a : b; }

int drot_ref_info_len(void) { return I_NINFO; }

/* Threads the sweep uses (1 without OpenMP). */
int drot_ref_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Step 4 and the sums of step 5 on rows [i0, i1): X_{k+1} written in place,
 * row sums to u[i], column sums of these rows to v (n entries), and the
 * partial <C, X_{k+1}> and r_dual^2 (at the incoming shifts) to out[0], out[1]. */
static void sweep_rows(long long i0, long long i1, long long n, const double *C,
                       const double *phi, const double *psi, double rho, double *X,
                       double *u, double *v, double *out) {
  double rd2 = 0.0, cost = 0.0;
  for (long long j = 0; j < n; ++j) v[j] = 0.0;
  for (long long i = i0; i < i1; ++i) {
    u[i] = 0.0;
    for (long long j = 0; j < n; ++j) {
      const double c = C[i * n + j];
      const double d = phi[i] / rho + psi[j] / rho - c;
      if (d > 0) rd2 += d * d;
      double x = X[i * n + j] + phi[i] + psi[j] - rho * c;
      if (!(x > 0)) x = 0.0;
      X[i * n + j] = x;
      u[i] += x;
      v[j] += x;
      cost += c * x;
    }
  }
  out[0] = cost;
  out[1] = rd2;
}

/*
 * Run DROT for at most max_iter iterations.
 *   C      (m*n)  cost, row-major, ld = n
 *   p (m), q (n)  marginals (equal total mass is the caller's duty)
 *   X      (m*n)  in: X_0 if x0_given, else ignored; out: X_K
 *   phi0/psi0     optional initial shifts (NULL = 0)
 *   phi/psi       out: phi_K (m), psi_K (n)
 *   a_out/b_out   optional out: a_K (m), b_K (n)
 *   info          out: I_NINFO doubles (see enum)
 *   trace         optional out: 6 doubles per iteration k = 1..K, rows
 *                 (pobj, dobj, r_primal, r_dual_lagged, gap, max_eps),
 *                 at most trace_cap rows.
 * Returns REF_OK (stopping test met), REF_MAXITER, or a negative error.
 */
int drot_ref_solve(long long m, long long n, const double *C, const double *p,
                   const double *q, double rho, double tol, int tol_mode,
                   long long max_iter, int x0_given, const double *phi0,
                   const double *psi0, double *X, double *phi, double *psi,
                   double *a_out, double *b_out, double *info, double *trace,
                   long long trace_cap) {
  if (m <= 0 || n <= 0 || !(rho > 0) || !(tol >= 0) || max_iter < 0) return REF_EINVAL;
  double *a = malloc(sizeof(double) * m), *b = malloc(sizeof(double) * n);
  double *u = malloc(sizeof(double) * m), *v = malloc(sizeof(double) * n);
  double *r = malloc(sizeof(double) * m), *s = malloc(sizeof(double) * n);
  double *phin = malloc(sizeof(double) * m), *psin = malloc(sizeof(double) * n);
  const int T = drot_ref_threads();
  double *vpart = malloc(sizeof(double) * (size_t)n * (size_t)T);
  double *spart = malloc(sizeof(double) * 2 * (size_t)T);
  if (!a || !b || !u || !v || !r || !s || !phin || !psin || !vpart || !spart) {
    free(a); free(b); free(u); free(v); free(r); free(s); free(phin); free(psin);
    free(vpart); free(spart);
    return REF_ENOMEM;
  }
  int nt = 1;
  const double mn = (double)(m + n);

  /* Step 1: X_0 (p q^T unless given) and the initial shifts. */
  if (!x0_given)
    for (long long i = 0; i < m; ++i)
      for (long long j = 0; j < n; ++j) X[i * n + j] = p[i] * q[j];
  for (long long i = 0; i < m; ++i) phi[i] = phi0 ? phi0[i] : 0.0;
  for (long long j = 0; j < n; ++j) psi[j] = psi0 ? psi0[j] : 0.0;

  /* Step 2: a_0 = Y_0 e - p, b_0 = Y_0^T f - q, alpha_0 = f^T a_0 / (m+n). */
  double sphi = 0.0, spsi = 0.0;
  for (long long i = 0; i < m; ++i) sphi += phi[i];
  for (long long j = 0; j < n; ++j) spsi += psi[j];
  for (long long i = 0; i < m; ++i) u[i] = 0.0;
  for (long long j = 0; j < n; ++j) v[j] = 0.0;
  for (long long i = 0; i < m; ++i)
    for (long long j = 0; j < n; ++j) {
      u[i] += X[i * n + j];
      v[j] += X[i * n + j];
    }
  for (long long i = 0; i < m; ++i) a[i] = u[i] - p[i] + (double)n * phi[i] + spsi;
  for (long long j = 0; j < n; ++j) b[j] = v[j] - q[j] + (double)m * psi[j] + sphi;
  double alpha = 0.0;
  for (long long i = 0; i < m; ++i) alpha += a[i];
  alpha /= mn;

  /* Scales for the relative stopping test. */
  double normC = 0.0, normpq = 0.0;
  for (long long k = 0; k < m * n; ++k) normC += C[k] * C[k];
  normC = sqrt(normC);
  for (long long i = 0; i < m; ++i) normpq += p[i] * p[i];
  for (long long j = 0; j < n; ++j) normpq += q[j] * q[j];
  normpq = sqrt(normpq);

  int status = REF_MAXITER;
  long long k = 0;
  double pobj = 0, dobj = 0, rp = 0, rd = 0, gap = 0, ep = 0, ed = 0, eg = 0;
  for (k = 0; k < max_iter;) {
    /* Step 4: X_{k+1} = [X_k + phi_k e^T + f psi_k^T - rho C]_+ ;
     * r_dual at (phi_k, psi_k) from the same read of C;
     * Step 5 sums u = X_{k+1} e, v = X_{k+1}^T f and <C, X_{k+1}>. */
#ifdef _OPENMP
#pragma omp parallel num_threads(T)
    {
      const int t = omp_get_thread_num(), tn = omp_get_num_threads();
#pragma omp single
      nt = tn;
      sweep_rows(m * t / tn, m * (t + 1) / tn, n, C, phi, psi, rho, X, u,
                 vpart + (size_t)t * (size_t)n, spart + 2 * t);
    }
#else
    sweep_rows(0, m, n, C, phi, psi, rho, X, u, vpart, spart);
#endif
    double cost = 0.0, rd2 = 0.0;
    for (long long j = 0; j < n; ++j) v[j] = 0.0;
    for (int t = 0; t < nt; ++t) {
      for (long long j = 0; j < n; ++j) v[j] += vpart[(size_t)t * (size_t)n + j];
      cost += spart[2 * t];
      rd2 += spart[2 * t + 1];
    }
    /* Step 5: residuals and beta. */
    double sr = 0.0, nr2 = 0.0, ns2 = 0.0;
    for (long long i = 0; i < m; ++i) {
      r[i] = u[i] - p[i];
      sr += r[i];
      nr2 += r[i] * r[i];
    }
    for (long long j = 0; j < n; ++j) {
      s[j] = v[j] - q[j];
      ns2 += s[j] * s[j];
    }
    const double beta = sr / mn;
    /* Steps 6-7: new shifts from the OLD a, b, alpha. */
    for (long long i = 0; i < m; ++i)
      phin[i] = (a[i] - 2.0 * r[i] + (2.0 * beta - alpha)) / (double)n;
    for (long long j = 0; j < n; ++j)
      psin[j] = (b[j] - 2.0 * s[j] + (2.0 * beta - alpha)) / (double)m;
    /* Step 8: accumulators. */
    for (long long i = 0; i < m; ++i) a[i] -= r[i];
    for (long long j = 0; j < n; ++j) b[j] -= s[j];
    alpha -= beta;
    memcpy(phi, phin, sizeof(double) * m);
    memcpy(psi, psin, sizeof(double) * n);
    ++k;

    /* Stopping criteria at iterate k (r_dual lagged by one iteration). */
    double pd = 0.0;
    for (long long i = 0; i < m; ++i) pd += p[i] * phi[i];
    for (long long j = 0; j < n; ++j) pd += q[j] * psi[j];
    pobj = cost;
    dobj = pd / rho;
    gap = fabs(pobj - dobj);
    rp = sqrt(nr2 + ns2);
    rd = sqrt(rd2);
    ep = rp / maxd(normpq, 1e-300);
    ed = rd / maxd(normC, 1e-300);
    eg = gap / maxd(maxd(fabs(pobj), fabs(dobj)), 1e-300);
    const double me = maxd(ep, maxd(ed, eg));
    const double ma = maxd(rp, maxd(rd, gap));
    if (trace && k <= trace_cap) {
      double *t = trace + 6 * (k - 1);
      t[0] = pobj; t[1] = dobj; t[2] = rp; t[3] = rd; t[4] = gap;
      t[5] = tol_mode ? ma : me;
    }
    if ((tol_mode ? ma : me) <= tol) {
      status = REF_OK;
      break;
    }
  }

  if (a_out) memcpy(a_out, a, sizeof(double) * m);
  if (b_out) memcpy(b_out, b, sizeof(double) * n);
  info[I_ITERS] = (double)k;
  info[I_STATUS] = (double)status;
  info[I_POBJ] = pobj;
  info[I_DOBJ] = dobj;
  info[I_RP] = rp;
  info[I_RD] = rd;
  info[I_GAP] = gap;
  info[I_EPS_P] = ep;
  info[I_EPS_D] = ed;
  info[I_EPS_G] = eg;
  info[I_ALPHA] = alpha;
  info[I_NORMC] = normC;
  info[I_NORMPQ] = normpq;
  free(a); free(b); free(u); free(v); free(r); free(s); free(phin); free(psin);
  free(vpart); free(spart);
  return status;
}

/*
 * Exact residuals of a given primal-dual pair (X, mu = phi/rho, nu = psi/rho):
 * r_primal, r_dual and the gap of the stopping criteria, all at the SAME
 * shifts (no lag), plus the primal and dual objectives.  info as above
 * (I_ITERS, I_STATUS, I_ALPHA are left 0).
 */
int drot_ref_eval(long long m, long long n, const double *C, const double *p,
                  const double *q, double rho, const double *X, const double *phi,
                  const double *psi, double *info) {
  if (m <= 0 || n <= 0 || !(rho > 0)) return REF_EINVAL;
  double *u = calloc((size_t)m, sizeof(double)), *v = calloc((size_t)n, sizeof(double));
  if (!u || !v) { free(u); free(v); return REF_ENOMEM; }
  double cost = 0.0, rd2 = 0.0, normC = 0.0, normpq = 0.0;
  for (long long i = 0; i < m; ++i)
    for (long long j = 0; j < n; ++j) {
      const double c = C[i * n + j], x = X[i * n + j];
      u[i] += x;
      v[j] += x;
      cost += c * x;
      const double d = phi[i] / rho + psi[j] / rho - c;
      if (d > 0) rd2 += d * d;
      normC += c * c;
    }
  double nr2 = 0.0, ns2 = 0.0, pd = 0.0;
  for (long long i = 0; i < m; ++i) {
    nr2 += (u[i] - p[i]) * (u[i] - p[i]);
    pd += p[i] * phi[i];
    normpq += p[i] * p[i];
  }
  for (long long j = 0; j < n; ++j) {
    ns2 += (v[j] - q[j]) * (v[j] - q[j]);
    pd += q[j] * psi[j];
    normpq += q[j] * q[j];
  }
  normC = sqrt(normC);
  normpq = sqrt(normpq);
  for (int t = 0; t < I_NINFO; ++t) info[t] = 0.0;
  info[I_POBJ] = cost;
  info[I_DOBJ] = pd / rho;
  info[I_RP] = sqrt(nr2 + ns2);
  info[I_RD] = sqrt(rd2);
  info[I_GAP] = fabs(info[I_POBJ] - info[I_DOBJ]);
  info[I_EPS_P] = info[I_RP] / maxd(normpq, 1e-300);
  info[I_EPS_D] = info[I_RD] / maxd(normC, 1e-300);
  info[I_EPS_G] = info[I_GAP] / maxd(maxd(fabs(info[I_POBJ]), fabs(info[I_DOBJ])), 1e-300);
  info[I_NORMC] = normC;
  info[I_NORMPQ] = normpq;
  free(u); free(v);
  return REF_OK;
}
