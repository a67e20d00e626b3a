// Contact solver for gfx950: projected Gauss-Seidel (PGS) on a batch of
// independent mixed linear complementarity problems, and its adjoint.
//
// Problem (Sec. 4.1 "Collision resolution", Eq. mlcp; App. C): find x with
//   a = A x + b,  lo <= x <= hi,  a_i >= 0 where x_i = lo_i,
//   a_i <= 0 where x_i = hi_i,  a_i = 0 in between,
// by niter sweeps from a start x0; each sweep sets the rows in order,
//   y_i = -(b_i + sum_{j != i} A_ij x_j) / A_ii,  x_i = min(max(y_i, lo_i), hi_i).
// The adjoint reverses the sweeps (App. C: the reverse solver mirrors the
// forward one with the adjoint of every operation) from the vector stored
// at the start of every sweep: the clamp sends x_bar_i to the active bound
// or to y_bar_i, then b_bar_i, A_bar_i. and x_bar_j (j != i) follow from
// y_i, and x_bar_i is reset.
//
// Layout on the GPU: one lane per problem.  A problem of n <= 16 rows is
// held in registers (A, and in the adjoint A_bar as well up to 12 rows) by a
// kernel compiled for NMAX rows (4, 8, 12 or 16; rows past n are skipped), so
// the row and column loops are unrolled and every operand has a fixed
// register.
// The sweep vectors go to the workspace as [niter + 1][n][batch], one
// coalesced row per wave and entry.  Problems are independent: no
// cross-lane traffic, no barriers.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/abadj.h"
#include "abadj_internal.h"

namespace {

constexpr int kBlock = 256;

template <typename S>
struct PgsArgs {
  int batch, n, niter;
  const S* A;    // [batch][n][n]
  const S* b;    // [batch][n]
  const S* lo;
  const S* hi;
  const S* x0;
  S* x;          // solve: result [batch][n]
  S* ws;         // nullable (solve) / required (adjoint): [niter + 1][n][batch]
  const S* xbar; // adjoint: seed [batch][n]
  S* Abar;       // adjoint outputs
  S* bbar;
  S* lobar;
  S* hibar;
  S* x0bar;
};

template <typename S, int N>
__global__ __launch_bounds__(kBlock) void k_pgs_solve(PgsArgs<S> P) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= P.batch) return;
  const int n = P.n;
  const size_t B = (size_t)P.batch;
  S A[N][N], b[N], lo[N], hi[N], x[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int j = 0; j < N; ++j) A[i][j] = (i < n && j < n) ? P.A[((size_t)p * n + i) * n + j] : S(0);
    b[i] = (i < n) ? P.b[(size_t)p * n + i] : S(0);
    lo[i] = (i < n) ? P.lo[(size_t)p * n + i] : S(0);
    hi[i] = (i < n) ? P.hi[(size_t)p * n + i] : S(0);
    x[i] = (i < n) ? P.x0[(size_t)p * n + i] : S(0);
  }
  for (int t = 0; t < P.niter; ++t) {
    if (P.ws) {
#pragma unroll
      for (int i = 0; i < N; ++i)
        if (i < n) P.ws[((size_t)t * n + i) * B + p] = x[i];
    }
#pragma unroll
    for (int i = 0; i < N; ++i) {
      if (i < n) {
        S d = S(0);
#pragma unroll
        for (int j = 0; j < N; ++j)
          if (j != i) d += A[i][j] * x[j];
        const S y = -(b[i] + d) / A[i][i];
        x[i] = (y < lo[i]) ? lo[i] : ((y > hi[i]) ? hi[i] : y);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < N; ++i)
    if (i < n) {
      P.x[(size_t)p * n + i] = x[i];
      if (P.ws) P.ws[((size_t)P.niter * n + i) * B + p] = x[i];
    }
}

template <typename S, int N>
__global__ __launch_bounds__(kBlock) void k_pgs_adjoint(PgsArgs<S> P) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= P.batch) return;
  const int n = P.n;
  const size_t B = (size_t)P.batch;
  S A[N][N], Ab[N][N], b[N], lo[N], hi[N], xb[N], bb[N], lb[N], hb[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
      A[i][j] = (i < n && j < n) ? P.A[((size_t)p * n + i) * n + j] : S(0);
      Ab[i][j] = S(0);
    }
    b[i] = (i < n) ? P.b[(size_t)p * n + i] : S(0);
    lo[i] = (i < n) ? P.lo[(size_t)p * n + i] : S(0);
    hi[i] = (i < n) ? P.hi[(size_t)p * n + i] : S(0);
    xb[i] = (i < n) ? P.xbar[(size_t)p * n + i] : S(0);
    bb[i] = lb[i] = hb[i] = S(0);
  }
  for (int t = P.niter - 1; t >= 0; --t) {
    // x at the start (xs) and the end (xe) of sweep t; before row i the
    // vector holds xe[j] for j < i and xs[j] for j > i
    S xs[N], xe[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      xs[j] = (j < n) ? P.ws[((size_t)t * n + j) * B + p] : S(0);
      xe[j] = (j < n) ? P.ws[((size_t)(t + 1) * n + j) * B + p] : S(0);
    }
#pragma unroll
    for (int i = N - 1; i >= 0; --i) {
      if (i < n) {
        S d = S(0);
#pragma unroll
        for (int j = 0; j < N; ++j)
          if (j != i) d += A[i][j] * ((j < i) ? xe[j] : xs[j]);
        const S y = -(b[i] + d) / A[i][i];
        S yb = S(0);
        if (y < lo[i]) lb[i] += xb[i];
        else if (y > hi[i]) hb[i] += xb[i];
        else yb = xb[i];
        xb[i] = S(0);
        const S db = -yb / A[i][i];
        bb[i] += db;
        Ab[i][i] += db * y;
#pragma unroll
        for (int j = 0; j < N; ++j)
          if (j != i) {
            Ab[i][j] += db * ((j < i) ? xe[j] : xs[j]);
            xb[j] += db * A[i][j];
          }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < N; ++i)
    if (i < n) {
#pragma unroll
      for (int j = 0; j < N; ++j)
        if (j < n) P.Abar[((size_t)p * n + i) * n + j] = Ab[i][j];
      P.bbar[(size_t)p * n + i] = bb[i];
      P.lobar[(size_t)p * n + i] = lb[i];
      P.hibar[(size_t)p * n + i] = hb[i];
      P.x0bar[(size_t)p * n + i] = xb[i];
    }
}

// The adjoint for the largest row bucket.  A and A_bar together (2 * 16^2
// per lane) do not fit the registers next to the vectors, so A_bar is formed
// in a second phase: the reverse sweeps keep A, the diagonal of A_bar and
// the vectors, and write each row's y_bar / (-A_ii) = db_{t,i} to the
// workspace after the sweep vectors; then, since
//   A_bar_ij = sum_t db_{t,i} x_j(t, i)  (j != i),
// with x_j(t, i) the value row i read in sweep t (the end-of-sweep value for
// j < i, the start-of-sweep one for j > i), RC rows of A_bar at a time are
// summed from db and the sweep vectors.  Each lane reads back only what it
// wrote itself.
constexpr int kSplitRows = 13;  // row counts from this up take the split adjoint
constexpr int kRC = 8;          // rows of A_bar per pass of the second phase

template <typename S, int N>
__global__ __launch_bounds__(kBlock) void k_pgs_adjoint_split(PgsArgs<S> P) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= P.batch) return;
  const int n = P.n;
  const size_t B = (size_t)P.batch;
  S* db = P.ws + (size_t)(P.niter + 1) * n * B;  // [niter][n][batch]
  S A[N][N], Ad[N], b[N], lo[N], hi[N], xb[N], bb[N], lb[N], hb[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int j = 0; j < N; ++j) A[i][j] = (i < n && j < n) ? P.A[((size_t)p * n + i) * n + j] : S(0);
    Ad[i] = S(0);
    b[i] = (i < n) ? P.b[(size_t)p * n + i] : S(0);
    lo[i] = (i < n) ? P.lo[(size_t)p * n + i] : S(0);
    hi[i] = (i < n) ? P.hi[(size_t)p * n + i] : S(0);
    xb[i] = (i < n) ? P.xbar[(size_t)p * n + i] : S(0);
    bb[i] = lb[i] = hb[i] = S(0);
  }
  for (int t = P.niter - 1; t >= 0; --t) {
    S xs[N], xe[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      xs[j] = (j < n) ? P.ws[((size_t)t * n + j) * B + p] : S(0);
      xe[j] = (j < n) ? P.ws[((size_t)(t + 1) * n + j) * B + p] : S(0);
    }
#pragma unroll
    for (int i = N - 1; i >= 0; --i) {
      if (i < n) {
        S d = S(0);
#pragma unroll
        for (int j = 0; j < N; ++j)
          if (j != i) d += A[i][j] * ((j < i) ? xe[j] : xs[j]);
        const S y = -(b[i] + d) / A[i][i];
        S yb = S(0);
        if (y < lo[i]) lb[i] += xb[i];
        else if (y > hi[i]) hb[i] += xb[i];
        else yb = xb[i];
        xb[i] = S(0);
        const S dbi = -yb / A[i][i];
        bb[i] += dbi;
        Ad[i] += dbi * y;
        db[((size_t)t * n + i) * B + p] = dbi;
#pragma unroll
        for (int j = 0; j < N; ++j)
          if (j != i) xb[j] += dbi * A[i][j];
      }
    }
  }
#pragma unroll
  for (int i = 0; i < N; ++i)
    if (i < n) {
      P.bbar[(size_t)p * n + i] = bb[i];
      P.lobar[(size_t)p * n + i] = lb[i];
      P.hibar[(size_t)p * n + i] = hb[i];
      P.x0bar[(size_t)p * n + i] = xb[i];
    }
  // second phase: the off-diagonal entries of A_bar, kRC rows at a time
#pragma unroll 1
  for (int r0 = 0; r0 < n; r0 += kRC) {
    S acc[kRC][N];
#pragma unroll
    for (int r = 0; r < kRC; ++r)
#pragma unroll
      for (int j = 0; j < N; ++j) acc[r][j] = S(0);
    for (int t = 0; t < P.niter; ++t) {
      S xs[N], xe[N];
#pragma unroll
      for (int j = 0; j < N; ++j) {
        xs[j] = (j < n) ? P.ws[((size_t)t * n + j) * B + p] : S(0);
        xe[j] = (j < n) ? P.ws[((size_t)(t + 1) * n + j) * B + p] : S(0);
      }
#pragma unroll
      for (int r = 0; r < kRC; ++r) {
        const int i = r0 + r;
        if (i < n) {
          const S dbi = db[((size_t)t * n + i) * B + p];
#pragma unroll
          for (int j = 0; j < N; ++j) acc[r][j] += dbi * ((j < i) ? xe[j] : xs[j]);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < kRC; ++r) {
      const int i = r0 + r;
      if (i < n) {
#pragma unroll
        for (int j = 0; j < N; ++j) {
          if (j < n) {
            // the diagonal is y's own term from the first phase
            S v = acc[r][j];
#pragma unroll
            for (int k = 0; k < N; ++k)
              if (k == i && j == k) v = Ad[k];
            P.Abar[((size_t)p * n + i) * n + j] = v;
          }
        }
      }
    }
  }
}

int pgs_fail(int code, const std::string& msg) { return aba::report_error(code, msg); }

// the sweep vectors [niter + 1][n][batch], and for the split adjoint's rows
// db [niter][n][batch] after them
size_t pgs_ws_bytes(int dtype, int batch, int n, int niter) {
  const size_t rows = (size_t)(niter + 1) + (n >= kSplitRows ? (size_t)niter : 0);
  return rows * (size_t)n * (size_t)batch * (dtype == SIM_F64 ? sizeof(double) : sizeof(float));
}

int pgs_check(const char* who, int dtype, int batch, int n, int niter) {
  if (dtype != SIM_F32 && dtype != SIM_F64)
    return pgs_fail(SIM_ERR_UNSUPPORTED_DTYPE, std::string(who) + ": dtype must be SIM_F32 or SIM_F64");
  if (batch < 0 || niter < 0 || n < 1 || n > SIM_PGS_MAX_ROWS)
    return pgs_fail(SIM_ERR_INVALID_ARG, std::string(who) + ": need batch >= 0, niter >= 0 and 1 <= n <= " +
                                             std::to_string(SIM_PGS_MAX_ROWS));
  return SIM_OK;
}

// one kernel per row bucket NMAX (4, 8, 12, 16); the largest bucket's
// adjoint is the split one
template <typename S, int N>
void launch_n(const PgsArgs<S>& a, hipStream_t st, bool adjoint, dim3 grid) {
  static_assert(N < kSplitRows || N == 16, "row buckets");
  if (adjoint) {
    if constexpr (N >= kSplitRows) hipLaunchKernelGGL((k_pgs_adjoint_split<S, N>), grid, dim3(kBlock), 0, st, a);
    else hipLaunchKernelGGL((k_pgs_adjoint<S, N>), grid, dim3(kBlock), 0, st, a);
  } else {
    hipLaunchKernelGGL((k_pgs_solve<S, N>), grid, dim3(kBlock), 0, st, a);
  }
}
template <typename S>
hipError_t launch(const PgsArgs<S>& a, hipStream_t st, bool adjoint) {
  if (a.batch == 0) return hipSuccess;
  const dim3 grid((a.batch + kBlock - 1) / kBlock);
  if (a.n <= 4) launch_n<S, 4>(a, st, adjoint, grid);
  else if (a.n <= 8) launch_n<S, 8>(a, st, adjoint, grid);
  else if (a.n <= 12) launch_n<S, 12>(a, st, adjoint, grid);
  else launch_n<S, 16>(a, st, adjoint, grid);
  return hipGetLastError();
}

}  // namespace

extern "C" {

int sim_pgs_workspace_bytes(int dtype, int batch, int n, int niter, size_t* bytes) {
  aba::clear_error();
  if (!bytes) return pgs_fail(SIM_ERR_INVALID_ARG, "sim_pgs_workspace_bytes: null argument");
  const int rc = pgs_check("sim_pgs_workspace_bytes", dtype, batch, n, niter);
  if (rc) return rc;
  *bytes = pgs_ws_bytes(dtype, batch, n, niter);
  return SIM_OK;
}

int sim_pgs_solve(int dtype, int batch, int n, int niter, const void* A, const void* b, const void* lo,
                  const void* hi, const void* x0, void* x, void* workspace, size_t workspace_bytes, void* stream) {
  aba::clear_error();
  int rc = pgs_check("sim_pgs_solve", dtype, batch, n, niter);
  if (rc) return rc;
  if (batch > 0 && (!A || !b || !lo || !hi || !x0 || !x))
    return pgs_fail(SIM_ERR_INVALID_ARG, "sim_pgs_solve: null array argument");
  if (workspace && workspace_bytes < pgs_ws_bytes(dtype, batch, n, niter))
    return pgs_fail(SIM_ERR_WORKSPACE_TOO_SMALL, "sim_pgs_solve: workspace of " + std::to_string(workspace_bytes) +
                                                     " bytes, need " +
                                                     std::to_string(pgs_ws_bytes(dtype, batch, n, niter)));
  hipError_t e;
  if (dtype == SIM_F64) {
    PgsArgs<double> a{batch, n, niter, (const double*)A, (const double*)b, (const double*)lo, (const double*)hi,
                      (const double*)x0, (double*)x, (double*)workspace, nullptr, nullptr, nullptr, nullptr,
                      nullptr, nullptr};
    e = launch<double>(a, (hipStream_t)stream, false);
  } else {
    PgsArgs<float> a{batch, n, niter, (const float*)A, (const float*)b, (const float*)lo, (const float*)hi,
                     (const float*)x0, (float*)x, (float*)workspace, nullptr, nullptr, nullptr, nullptr,
                     nullptr, nullptr};
    e = launch<float>(a, (hipStream_t)stream, false);
  }
  if (e != hipSuccess) return pgs_fail(SIM_ERR_HIP, std::string("sim_pgs_solve: launch failed: ") + hipGetErrorString(e));
  return SIM_OK;
}

int sim_pgs_adjoint(int dtype, int batch, int n, int niter, const void* A, const void* b, const void* lo,
                    const void* hi, const void* xbar, void* workspace, size_t workspace_bytes, void* Abar,
                    void* bbar, void* lobar, void* hibar, void* x0bar, void* stream) {
  aba::clear_error();
  int rc = pgs_check("sim_pgs_adjoint", dtype, batch, n, niter);
  if (rc) return rc;
  if (batch > 0 && (!A || !b || !lo || !hi || !xbar || !workspace || !Abar || !bbar || !lobar || !hibar || !x0bar))
    return pgs_fail(SIM_ERR_INVALID_ARG, "sim_pgs_adjoint: null array argument");
  if (workspace_bytes < pgs_ws_bytes(dtype, batch, n, niter))
    return pgs_fail(SIM_ERR_WORKSPACE_TOO_SMALL, "sim_pgs_adjoint: workspace of " +
                                                     std::to_string(workspace_bytes) + " bytes, need " +
                                                     std::to_string(pgs_ws_bytes(dtype, batch, n, niter)));
  hipError_t e;
  if (dtype == SIM_F64) {
    PgsArgs<double> a{batch, n, niter, (const double*)A, (const double*)b, (const double*)lo, (const double*)hi,
                      nullptr, nullptr, (double*)workspace, (const double*)xbar, (double*)Abar, (double*)bbar,
                      (double*)lobar, (double*)hibar, (double*)x0bar};
    e = launch<double>(a, (hipStream_t)stream, true);
  } else {
    PgsArgs<float> a{batch, n, niter, (const float*)A, (const float*)b, (const float*)lo, (const float*)hi,
                     nullptr, nullptr, (float*)workspace, (const float*)xbar, (float*)Abar, (float*)bbar,
                     (float*)lobar, (float*)hibar, (float*)x0bar};
    e = launch<float>(a, (hipStream_t)stream, true);
  }
  if (e != hipSuccess)
    return pgs_fail(SIM_ERR_HIP, std::string("sim_pgs_adjoint: launch failed: ") + hipGetErrorString(e));
  return SIM_OK;
}

}  // extern "C"
