// Per-mode helpers of the Fourier-space fluid update (shared by the update kernel and the last
// products pass that performs the update itself).
#pragma once

#include "plan.hpp"

namespace fsib {

struct ModeGeo {
  int dim;
  int64_t N[3];
  int64_t Hx;
  double L;
};

__device__ __forceinline__ int64_t mode_of(int64_t i, int64_t n) { return i < (n + 1) / 2 ? i : i - n; }

__device__ __forceinline__ int sym_index(int a, int b, int dim) {
  if (a > b) {
    const int t = a;
    a = b;
    b = t;
  }
  if (dim == 3) {
    const int base[3] = {0, 3, 5};
    return base[a] + (b - a);
  }
  return a == 0 ? b : 2;
}

// Navier-Stokes update of one mode (Alg. 1 with V-hat of Alg. 2): P = fhat/rho - shat (plus the
// uniform body force at k = 0), Q = P - k (k.P)/|k|^2 with |k|^2 := 1 at k = 0 (projection only),
// half step u_mid = (dt/2 Q + u)/(1 + a), full step u_new = (dt Q + (1 - a) u)/(1 + a),
// a = mu dt |k|^2 / (2 rho) with the true |k|^2.  s[a] is shat_a = sum_b i k_b (u_a u_b)^.
template <typename T, int DIM>
__device__ __forceinline__ void ns_mode_update(int mode, T rho, T mu, T dt, const T* body, const T* k, T k2,
                                               const cplx<T>* s, const cplx<T>* f, const cplx<T>* u, cplx<T>* r) {
  cplx<T> P[3];
  cplx<T> kP = mk((T)0, (T)0);
  const T inv_rho = (T)1 / rho;
  for (int a = 0; a < DIM; ++a) {
    P[a] = f[a] * inv_rho - s[a];
    if (k2 == (T)0) P[a].x += body[a] * inv_rho;  // uniform body force
    kP = kP + P[a] * k[a];
  }
  const T k2p = k2 == (T)0 ? (T)1 : k2;
  const T av = mu * dt * k2 / ((T)2 * rho);
  const T den = (T)1 / ((T)1 + av);
  for (int a = 0; a < DIM; ++a) {
    const cplx<T> Q = P[a] - kP * (k[a] / k2p);
    if (mode == FLUID_NS_HALF)
      r[a] = (Q * (dt * (T)0.5) + u[a]) * den;
    else
      r[a] = (Q * dt + u[a] * ((T)1 - av)) * den;
  }
}

}  // namespace fsib
