// Internal launch interface between the host runtime and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace aba {

constexpr int kWave = 64;

// integer per-lane fields, stored [field][slot]
enum CiField { CI_PARENT = 0, CI_DEPTH, CI_CFIRST, CI_CCOUNT, CI_JTYPE, CI_QIDX, CI_VIDX, CI_UIDX, CI_COUNT };
// floating per-lane fields, stored [field][slot]
enum CfField {
  CF_ET = 0,          // 9
  CF_RT = 9,          // 3
  CF_AX = 12,         // 3
  CF_M = 15,          // 1
  CF_MC = 16,         // 3
  CF_IB = 19,         // 6: xx yy zz xy xz yz
  CF_COUNT = 25
};

template <typename S>
struct Packed {
  const int32_t* ci;     // [CI_COUNT][nslots]
  const S* cf;           // [CF_COUNT][nslots]
  const int32_t* wmaxd;  // [nwaves] deepest level present in each wave
  int nslots;
  int nwaves;
  S g[3];                // gravity
  int nq, nv, nu;        // totals over the batch
};

template <typename S>
struct FwdArgs {
  Packed<S> P;
  S dt;
  int T, K;
  const S* q0;
  const S* qd0;
  const S* tau;  // [T][nu]
  S* qT;
  S* qdT;
  S* traj;       // nullable [T][nq + nv]
  S* ck;         // nullable: checkpoints [ceil(T/K)][state width][nslots]
};

template <typename S>
struct BwdArgs {
  Packed<S> P;
  S dt;
  int T, K;
  const S* tau;
  const S* gqT;
  const S* gqdT;
  const S* gtraj;  // nullable
  S* gq0;
  S* gqd0;
  S* gtau;
  const S* ck;
  S* scratch;      // K > 1: [K][state width][nslots]
};

template <typename S>
struct AbaArgs {
  Packed<S> P;
  const S* q;
  const S* qd;
  const S* tau;
  S* qdd;
};

// state width per lane slot in checkpoint / scratch arrays
constexpr int state_width(bool has_free) { return has_free ? 13 : 2; }

template <typename S>
hipError_t launch_forward(const FwdArgs<S>& a, bool has_free, hipStream_t st);
template <typename S>
hipError_t launch_backward(const BwdArgs<S>& a, bool has_free, hipStream_t st);
template <typename S>
hipError_t launch_aba(const AbaArgs<S>& a, bool has_free, hipStream_t st);

}  // namespace aba
