/*
 * Plain CPU oracle of the contact solver: projected Gauss-Seidel (PGS) on a
 * mixed linear complementarity problem and its adjoint.  TEST
 * INFRASTRUCTURE ONLY (tests, smoke check, benchmark CPU baseline).
 *
 * Problem (Sec. 4.1 "Collision resolution", Eq. mlcp; App. C): find x with
 *   a = A x + b,  lo <= x <= hi,  and for every row i
 *   a_i >= 0 where x_i = lo_i,  a_i <= 0 where x_i = hi_i,  a_i = 0 between;
 * with lo = 0 and hi = +inf this is 0 <= a  perp  x >= 0.  The solver runs a
 * fixed number of sweeps from a given start x0; each sweep visits the rows in
 * order and sets row i from the current values of the others:
 *   y_i = -(b_i + d_i) / A_ii,  d_i = sum_{j != i} A_ij x_j,
 *   x_i = min(max(y_i, lo_i), hi_i).
 * The printed listing of App. C is garbled (see the readings recorded with
 * the build); this follows the definition above.
 *
 * Adjoint (App. C: the reverse solver mirrors the forward one with the
 * adjoint of every operation, from the stored vectors of each sweep): the
 * forward pass keeps x at the start of every sweep, and the reverse visits
 * the sweeps backwards and, in each, the rows from the last to the first.
 * For row i the adjoint of the clamp sends x_bar_i to the active bound
 * (lo_bar_i or hi_bar_i) or to y_bar_i; then
 *   b_bar_i += -y_bar_i / A_ii,  A_bar_ii += -y_bar_i y_i / A_ii,
 *   A_bar_ij += (-y_bar_i / A_ii) x_j,  x_bar_j += (-y_bar_i / A_ii) A_ij,
 * and x_bar_i is reset (the row overwrote x_i).  What is left in x_bar at
 * the end is the adjoint of the start x0.
 *
 * Ties: the clamp is active when y_i < lo_i or y_i > hi_i strictly (a value
 * on a bound passes its adjoint through, the one-sided derivative from
 * inside the box).
 */
#include <complex.h>
#include <string.h>

#include "oracle.h"

static double clampd(double y, double lo, double hi, int *state) {
  if (y < lo) { *state = -1; return lo; }
  if (y > hi) { *state = 1; return hi; }
  *state = 0;
  return y;
}

void orc_pgs_solve(int n, int niter, const double *A, const double *b, const double *lo,
                   const double *hi, const double *x0, double *x, double *sweeps) {
  memcpy(x, x0, sizeof(double) * (size_t)n);
  for (int t = 0; t < niter; ++t) {
    if (sweeps) memcpy(sweeps + (size_t)t * n, x, sizeof(double) * (size_t)n);
    for (int i = 0; i < n; ++i) {
      double d = 0;
      for (int j = 0; j < n; ++j)
        if (j != i) d += A[(size_t)i * n + j] * x[j];
      const double y = -(b[i] + d) / A[(size_t)i * n + i];
      int st;
      x[i] = clampd(y, lo[i], hi[i], &st);
    }
  }
  if (sweeps) memcpy(sweeps + (size_t)niter * n, x, sizeof(double) * (size_t)n);
}

/* Complex-step version (tests): every input may carry an imaginary
 * perturbation; the clamp decides on real parts and passes the chosen
 * operand through whole, which extends the piecewise-linear map exactly
 * away from its kinks. */
void orc_pgs_solve_c(int n, int niter, const void *A_, const void *b_, const void *lo_,
                     const void *hi_, const void *x0_, void *x_) {
  const double complex *A = (const double complex *)A_, *b = (const double complex *)b_;
  const double complex *lo = (const double complex *)lo_, *hi = (const double complex *)hi_;
  double complex *x = (double complex *)x_;
  memcpy(x, x0_, sizeof(double complex) * (size_t)n);
  for (int t = 0; t < niter; ++t)
    for (int i = 0; i < n; ++i) {
      double complex d = 0;
      for (int j = 0; j < n; ++j)
        if (j != i) d += A[(size_t)i * n + j] * x[j];
      const double complex y = -(b[i] + d) / A[(size_t)i * n + i];
      if (creal(y) < creal(lo[i])) x[i] = lo[i];
      else if (creal(y) > creal(hi[i])) x[i] = hi[i];
      else x[i] = y;
    }
}

void orc_pgs_adjoint(int n, int niter, const double *A, const double *b, const double *lo,
                     const double *hi, const double *sweeps, const double *xbar_in, double *Abar,
                     double *bbar, double *lobar, double *hibar, double *x0bar) {
  for (size_t k = 0; k < (size_t)n * n; ++k) Abar[k] = 0;
  for (int i = 0; i < n; ++i) { bbar[i] = 0; lobar[i] = 0; hibar[i] = 0; }
  double xb[n], cur[n];
  memcpy(xb, xbar_in, sizeof(double) * (size_t)n);
  for (int t = niter - 1; t >= 0; --t) {
    const double *xs = sweeps + (size_t)t * n, *xe = sweeps + (size_t)(t + 1) * n;
    /* before row i of sweep t the vector holds xe[j] for j < i and xs[j] for j >= i */
    for (int i = n - 1; i >= 0; --i) {
      for (int j = 0; j < n; ++j) cur[j] = (j < i) ? xe[j] : xs[j];
      double d = 0;
      for (int j = 0; j < n; ++j)
        if (j != i) d += A[(size_t)i * n + j] * cur[j];
      const double Aii = A[(size_t)i * n + i];
      const double y = -(b[i] + d) / Aii;
      int st;
      (void)clampd(y, lo[i], hi[i], &st);
      double yb = 0;
      if (st < 0) lobar[i] += xb[i];
      else if (st > 0) hibar[i] += xb[i];
      else yb = xb[i];
      xb[i] = 0;
      const double db = -yb / Aii;
      bbar[i] += db;
      Abar[(size_t)i * n + i] += db * y;
      for (int j = 0; j < n; ++j)
        if (j != i) {
          Abar[(size_t)i * n + j] += db * cur[j];
          xb[j] += db * A[(size_t)i * n + j];
        }
    }
  }
  memcpy(x0bar, xb, sizeof(double) * (size_t)n);
}
