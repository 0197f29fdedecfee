// Building blocks of the transforms' adjoints (gradients; the adjoint of type-1 is type-2 and vice
// versa, App. A eqs. type1 and type2).  The position gradient of a sum needs the derivative of its
// phases, d/dx_a exp(+-i k.x) = +-i k_a exp(+-i k.x): a type-2 sum of an i k_a-weighted spectrum,
// combined per point with the strengths or with the incoming gradient.
#include "plan.hpp"

namespace fsib {

// out[c][k] = scale * (axis < 0 ? 1 : i k_axis) * in[c][k] for `count` spectral arrays of n0 x n1 x n2
// entries (x fastest).  Full spectra: entry i of an axis of length N is mode i, or i - N past the
// middle (FFT order).  Half spectra (x has n0 = N_x/2 + 1 entries): entry i along x is mode i.
template <typename T>
__global__ void k_spectral_scale(int64_t total, int n0, int n1, int n2, int nx_full, int axis, T kscale, T scale,
                                 const cplx<T>* __restrict__ in, cplx<T>* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const cplx<T> v = in[e];
  T f = scale;
  if (axis >= 0) {
    const int64_t cell = e % ((int64_t)n0 * n1 * n2);
    int m;
    if (axis == 0) {
      const int i = (int)(cell % n0);
      m = nx_full > 0 ? (i < (nx_full + 1) / 2 ? i : i - nx_full) : i;  // nx_full = 0: half spectrum
    } else if (axis == 1) {
      const int i = (int)((cell / n0) % n1);
      m = i < (n1 + 1) / 2 ? i : i - n1;
    } else {
      const int i = (int)(cell / ((int64_t)n0 * n1));
      m = i < (n2 + 1) / 2 ? i : i - n2;
    }
    f *= kscale * (T)m;
    out[e] = mk(-v.y * f, v.x * f);  // i f v
  } else {
    out[e] = v * f;
  }
}

// kind 0: gX[j][axis] = scale * sum_t Re( conj(u[t][j]) v[t][j] )      (u, v: ntr x M complex)
// kind 1: gX[j][axis] = scale * sum_a (u[j][a] v[j][a] + u2[j][a] v2[j][a])  (real (M, dim); u2, v2
//         may be null)
template <typename T>
__global__ void k_grad_combine(int64_t M, int kind, int ntr, int dim, int axis, double scale, const T* __restrict__ u,
                               const T* __restrict__ v, const T* __restrict__ u2, const T* __restrict__ v2,
                               double* __restrict__ gX) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  double s = 0.0;
  if (kind == 0) {
    for (int t = 0; t < ntr; ++t) {
      const int64_t q = 2 * ((int64_t)t * M + j);
      s += (double)u[q] * (double)v[q] + (double)u[q + 1] * (double)v[q + 1];
    }
  } else {
    for (int a = 0; a < dim; ++a) {
      s += (double)u[j * dim + a] * (double)v[j * dim + a];
      if (u2) s += (double)u2[j * dim + a] * (double)v2[j * dim + a];
    }
  }
  gX[j * dim + axis] = scale * s;
}

hipError_t launch_spectral_scale(const Plan& p, int layout, int axis, double scale, const void* in, void* out,
                                 hipStream_t st) {
  const int n0 = (int)(layout == 0 ? p.N[0] : p.Hx);
  const int64_t per = (int64_t)n0 * p.N[1] * p.N[2];
  const int64_t total = per * (layout == 0 ? p.ntrans : p.dim);
  if (total <= 0) return hipSuccess;
  const unsigned nblk = (unsigned)((total + 255) / 256);
  const double ks = 6.283185307179586476925286766559 / p.L;
  const int nxf = layout == 0 ? (int)p.N[0] : 0;
  if (p.prec == FSIB_F64)
    hipLaunchKernelGGL(k_spectral_scale<double>, dim3(nblk), dim3(256), 0, st, total, n0, (int)p.N[1], (int)p.N[2], nxf,
                       axis, ks, scale, (const cplx<double>*)in, (cplx<double>*)out);
  else
    hipLaunchKernelGGL(k_spectral_scale<float>, dim3(nblk), dim3(256), 0, st, total, n0, (int)p.N[1], (int)p.N[2], nxf,
                       axis, (float)ks, (float)scale, (const cplx<float>*)in, (cplx<float>*)out);
  return hipGetLastError();
}

hipError_t launch_grad_combine(const Plan& p, int64_t M, int kind, const void* u, const void* v, const void* u2,
                               const void* v2, double scale, double* gX, int axis, hipStream_t st) {
  if (M <= 0) return hipSuccess;
  const unsigned nblk = (unsigned)((M + 255) / 256);
  if (p.prec == FSIB_F64)
    hipLaunchKernelGGL(k_grad_combine<double>, dim3(nblk), dim3(256), 0, st, M, kind, p.ntrans, p.dim, axis, scale,
                       (const double*)u, (const double*)v, (const double*)u2, (const double*)v2, gX);
  else
    hipLaunchKernelGGL(k_grad_combine<float>, dim3(nblk), dim3(256), 0, st, M, kind, p.ntrans, p.dim, axis, scale,
                       (const float*)u, (const float*)v, (const float*)u2, (const float*)v2, gX);
  return hipGetLastError();
}

}  // namespace fsib
