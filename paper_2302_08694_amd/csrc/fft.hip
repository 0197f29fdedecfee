// Batched mixed-radix (2, 3, 4, 5) Stockham FFT passes in LDS.
//
// One pass transforms every line of one axis of a [outer][len][inner] complex array.  A
// workgroup loads `nb` lines into LDS (contiguous lines for the x axis; `nb` neighbouring columns
// for strided axes, so that global accesses stay coalesced), runs the Stockham stages between two
// LDS buffers, and stores.  Zero padding of the input and truncation of the output to a mode set
// in FFT order, and per-mode real factors (the NUFFT deconvolution, App. A eqs. type1_deco and
// type2_divi) are folded into the load and store, so pruned transforms read and write only the
// entries that exist.  Real-data passes along x pack two real lines into one complex line.
//
// Stockham stage (radix r, p = product of the radices already applied, m = n/r): butterfly i < m,
// k = i mod p, inputs x[i + q m] (q < r) twiddled by exp(sign 2 pi i q k / (p r)), outputs
// y[(i - k) r + k + q p].
#include "plan.hpp"

namespace fsib {

constexpr int kFftThreads = 256;

template <typename T>
__device__ __forceinline__ void bfly(int r, cplx<T>* u, T sg) {
  if (r == 2) {
    const cplx<T> a = u[0], b = u[1];
    u[0] = a + b;
    u[1] = a - b;
  } else if (r == 4) {
    const cplx<T> s02 = u[0] + u[2], d02 = u[0] - u[2], s13 = u[1] + u[3], d13 = u[1] - u[3];
    u[0] = s02 + s13;
    u[2] = s02 - s13;
    u[1] = d02 + mul_i(d13, sg);
    u[3] = d02 - mul_i(d13, sg);
  } else if (r == 3) {
    const T c = (T)-0.5, s = (T)0.86602540378443864676;
    const cplx<T> t = u[1] + u[2], d = u[1] - u[2];
    const cplx<T> a = u[0] + t * c;
    u[0] = u[0] + t;
    const cplx<T> b = mul_i(d, sg * s);
    u[1] = a + b;
    u[2] = a - b;
  } else {  // r == 5
    const T c1 = (T)0.30901699437494742410, c2 = (T)-0.80901699437494742410;
    const T s1 = (T)0.95105651629515357212, s2 = (T)0.58778525229247312917;
    const cplx<T> t1 = u[1] + u[4], t2 = u[2] + u[3], t3 = u[1] - u[4], t4 = u[2] - u[3];
    const cplx<T> a1 = u[0] + t1 * c1 + t2 * c2;
    const cplx<T> a2 = u[0] + t1 * c2 + t2 * c1;
    const cplx<T> b1 = mul_i(t3 * s1 + t4 * s2, sg);
    const cplx<T> b2 = mul_i(t3 * s2 - t4 * s1, sg);
    u[0] = u[0] + t1 + t2;
    u[1] = a1 + b1;
    u[4] = a1 - b1;
    u[2] = a2 + b2;
    u[3] = a2 - b2;
  }
}

// LDS index of entry t of line b: lines contiguous (x passes) or interleaved (strided passes).
template <bool CONTIG>
__device__ __forceinline__ int lidx(int t, int b, int n, int nb) {
  return CONTIG ? b * n + t : t * nb + b;
}

// Runs all Stockham stages on nb lines held in buf0; returns the buffer holding the result.
template <typename T, bool CONTIG>
__device__ cplx<T>* stockham(const FftArgs<T>& a, cplx<T>* buf0, cplx<T>* buf1) {
  const int n = a.n, nb = a.nb;
  const T sg = (T)a.sign;
  cplx<T>* src = buf0;
  cplx<T>* dst = buf1;
  int p = 1;
  for (int s = 0; s < a.nst; ++s) {
    const int r = a.radix[s];
    const int m = n / r;
    const int twstride = n / (p * r);
    for (int it = threadIdx.x; it < m * nb; it += kFftThreads) {
      int i, b;
      if (CONTIG) {
        b = it / m;
        i = it - b * m;
      } else {
        i = it / nb;
        b = it - i * nb;
      }
      const int k = i % p;
      cplx<T> u[5];
      for (int q = 0; q < r; ++q) u[q] = src[lidx<CONTIG>(i + q * m, b, n, nb)];
      if (p > 1) {
        for (int q = 1; q < r; ++q) {
          cplx<T> w = a.tw[q * k * twstride];
          if (a.sign > 0) w.y = -w.y;
          u[q] = cmul(u[q], w);
        }
      }
      bfly<T>(r, u, sg);
      const int j0 = (i - k) * r + k;
      for (int q = 0; q < r; ++q) dst[lidx<CONTIG>(j0 + q * p, b, n, nb)] = u[q];
    }
    __syncthreads();
    cplx<T>* tmp = src;
    src = dst;
    dst = tmp;
    p *= r;
  }
  return src;
}

template <typename T, bool CONTIG>
__global__ __launch_bounds__(kFftThreads) void k_fft_c2c(const cplx<T>* __restrict__ in, cplx<T>* __restrict__ out,
                                                         FftArgs<T> a) {
  extern __shared__ char smem_raw[];
  cplx<T>* buf0 = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* buf1 = buf0 + a.n * a.nb;
  const int n = a.n, nb = a.nb;
  int64_t o0 = 0, q0 = 0;
  int ncol;
  if (CONTIG) {
    o0 = (int64_t)blockIdx.x * nb;
    ncol = (int)(a.outer - o0 < nb ? a.outer - o0 : nb);
  } else {
    q0 = (int64_t)blockIdx.x * nb;
    o0 = blockIdx.y;
    ncol = (int)(a.inner - q0 < nb ? a.inner - q0 : nb);
  }
  // zero the padding gap [pin, n - (nin - pin))
  const int g0 = a.pin, g1 = n - (a.nin - a.pin);
  for (int it = threadIdx.x; it < (g1 - g0) * nb; it += kFftThreads) {
    int t, b;
    if (CONTIG) {
      b = it / (g1 - g0);
      t = g0 + it - b * (g1 - g0);
    } else {
      t = g0 + it / nb;
      b = it % nb;
    }
    buf0[lidx<CONTIG>(t, b, n, nb)] = mk((T)0, (T)0);
  }
  for (int it = threadIdx.x; it < a.nin * nb; it += kFftThreads) {
    int i, b;
    if (CONTIG) {
      b = it / a.nin;
      i = it - b * a.nin;
    } else {
      i = it / nb;
      b = it - i * nb;
    }
    const int t = i < a.pin ? i : n - (a.nin - i);
    cplx<T> v = mk((T)0, (T)0);
    if (b < ncol) {
      const int64_t gi = CONTIG ? (o0 + b) * a.nin + i : (o0 * a.nin + i) * a.inner + q0 + b;
      v = in[gi];
      if (a.fac_in) v = v * a.fac_in[i];
    }
    buf0[lidx<CONTIG>(t, b, n, nb)] = v;
  }
  __syncthreads();
  const cplx<T>* res = stockham<T, CONTIG>(a, buf0, buf1);
  for (int it = threadIdx.x; it < a.nout * nb; it += kFftThreads) {
    int i, b;
    if (CONTIG) {
      b = it / a.nout;
      i = it - b * a.nout;
    } else {
      i = it / nb;
      b = it - i * nb;
    }
    if (b >= ncol) continue;
    const int t = i < a.pout ? i : n - (a.nout - i);
    T f = a.scale;
    if (a.fac_out) f *= a.fac_out[i];
    const int64_t go = CONTIG ? (o0 + b) * a.nout + i : (o0 * a.nout + i) * a.inner + q0 + b;
    out[go] = res[lidx<CONTIG>(t, b, n, nb)] * f;
  }
}

// Real lines along x -> half spectra: lines 2b and 2b+1 form z = a + i b; A_m = (Z_m + conj Z_{n-m})/2,
// B_m = (Z_m - conj Z_{n-m})/(2i) for m < nout.  a.outer = number of real lines.
template <typename T>
__global__ __launch_bounds__(kFftThreads) void k_fft_r2c_x(const T* __restrict__ in, cplx<T>* __restrict__ out,
                                                           FftArgs<T> a) {
  extern __shared__ char smem_raw[];
  cplx<T>* buf0 = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* buf1 = buf0 + a.n * a.nb;
  const int n = a.n, nb = a.nb;
  const int64_t pair0 = (int64_t)blockIdx.x * nb;
  for (int it = threadIdx.x; it < n * nb; it += kFftThreads) {
    const int b = it / n, t = it - b * n;
    const int64_t r0 = 2 * (pair0 + b), r1 = r0 + 1;
    const T re = r0 < a.outer ? in[r0 * n + t] : (T)0;
    const T im = r1 < a.outer ? in[r1 * n + t] : (T)0;
    buf0[b * n + t] = mk(re, im);
  }
  __syncthreads();
  const cplx<T>* res = stockham<T, true>(a, buf0, buf1);
  for (int it = threadIdx.x; it < a.nout * nb; it += kFftThreads) {
    const int b = it / a.nout, m = it - b * a.nout;
    const int64_t r0 = 2 * (pair0 + b), r1 = r0 + 1;
    if (r0 >= a.outer) continue;
    const cplx<T> Z = res[b * n + m];
    const cplx<T> Zc = conj(res[b * n + (m == 0 ? 0 : n - m)]);
    T f = a.scale * (T)0.5;
    if (a.fac_out) f *= a.fac_out[m];
    const cplx<T> s = Z + Zc, d = Z - Zc;
    out[r0 * a.nout + m] = s * f;
    if (r1 < a.outer) out[r1 * a.nout + m] = mk(d.y * f, -d.x * f);
  }
}

// Half spectra along x (nin entries m = 0..nin-1, the rest zero) -> real lines of length n; two
// lines per complex transform: Z_t = A_t + i B_t with A_{n-m} = conj A_m, then Re/Im of the
// inverse transform.  a.outer = number of real lines.
template <typename T>
__global__ __launch_bounds__(kFftThreads) void k_fft_c2r_x(const cplx<T>* __restrict__ in, T* __restrict__ out,
                                                           FftArgs<T> a) {
  extern __shared__ char smem_raw[];
  cplx<T>* buf0 = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* buf1 = buf0 + a.n * a.nb;
  const int n = a.n, nb = a.nb;
  const int64_t pair0 = (int64_t)blockIdx.x * nb;
  for (int it = threadIdx.x; it < n * nb; it += kFftThreads) {
    const int b = it / n, t = it - b * n;
    const int64_t r0 = 2 * (pair0 + b), r1 = r0 + 1;
    const bool front = 2 * t <= n;
    const int m = front ? t : n - t;
    cplx<T> A = mk((T)0, (T)0), B = mk((T)0, (T)0);
    if (m < a.nin) {
      T f = (T)1;
      if (a.fac_in) f = a.fac_in[m];
      if (r0 < a.outer) A = in[r0 * a.nin + m] * f;
      if (r1 < a.outer) B = in[r1 * a.nin + m] * f;
      if (m == 0 || 2 * m == n) {
        A.y = (T)0;
        B.y = (T)0;
      } else if (!front) {
        A = conj(A);
        B = conj(B);
      }
    }
    buf0[b * n + t] = mk(A.x - B.y, A.y + B.x);
  }
  __syncthreads();
  const cplx<T>* res = stockham<T, true>(a, buf0, buf1);
  for (int it = threadIdx.x; it < n * nb; it += kFftThreads) {
    const int b = it / n, t = it - b * n;
    const int64_t r0 = 2 * (pair0 + b), r1 = r0 + 1;
    const cplx<T> z = res[b * n + t];
    if (r0 < a.outer) out[r0 * n + t] = z.x * a.scale;
    if (r1 < a.outer) out[r1 * n + t] = z.y * a.scale;
  }
}

template <typename T>
static FftArgs<T> base_args(const Plan& p, int n, int sign) {
  FftArgs<T> a;
  a.n = n;
  a.nst = radix_plan(n, a.radix);
  a.tw = (const cplx<T>*)p.tw.at(n);
  a.sign = sign;
  a.fac_in = nullptr;
  a.fac_out = nullptr;
  a.scale = (T)1;
  return a;
}

// LDS budget: two buffers of n*nb complex values within 64 KiB.
template <typename T>
static int lines_per_block(int n) {
  const int budget = (int)(32768 / sizeof(cplx<T>));  // complex entries per buffer
  int nb = budget / n;
  return nb < 1 ? 1 : (nb > 16 ? 16 : nb);
}

template <typename T>
static hipError_t c2c_impl(const Plan& p, const void* in, void* out, int n, int sign, int64_t inner, int64_t outer,
                           int nin, int pin, int nout, int pout, const void* fin, const void* fout, double scale,
                           hipStream_t st) {
  FftArgs<T> a = base_args<T>(p, n, sign);
  a.inner = inner;
  a.outer = outer;
  a.nin = nin;
  a.pin = pin;
  a.nout = nout;
  a.pout = pout;
  a.fac_in = (const T*)fin;
  a.fac_out = (const T*)fout;
  a.scale = (T)scale;
  int nb = lines_per_block<T>(n);
  if (inner == 1) {
    a.nb = nb;
    const size_t lds = 2 * (size_t)n * nb * sizeof(cplx<T>);
    hipLaunchKernelGGL((k_fft_c2c<T, true>), dim3((unsigned)((outer + nb - 1) / nb)), dim3(kFftThreads), lds, st,
                       (const cplx<T>*)in, (cplx<T>*)out, a);
  } else {
    if (nb > inner) nb = (int)inner;
    a.nb = nb;
    const size_t lds = 2 * (size_t)n * nb * sizeof(cplx<T>);
    hipLaunchKernelGGL((k_fft_c2c<T, false>), dim3((unsigned)((inner + nb - 1) / nb), (unsigned)outer),
                       dim3(kFftThreads), lds, st, (const cplx<T>*)in, (cplx<T>*)out, a);
  }
  return hipGetLastError();
}

hipError_t launch_fft_c2c(const Plan& p, const void* in, void* out, int n, int sign, int64_t inner, int64_t outer,
                          int nin, int pin, int nout, int pout, const void* fac_in, const void* fac_out, double scale,
                          hipStream_t st) {
  if (outer <= 0 || inner <= 0) return hipSuccess;
  return p.prec == FSIB_F64
             ? c2c_impl<double>(p, in, out, n, sign, inner, outer, nin, pin, nout, pout, fac_in, fac_out, scale, st)
             : c2c_impl<float>(p, in, out, n, sign, inner, outer, nin, pin, nout, pout, fac_in, fac_out, scale, st);
}

template <typename T>
static hipError_t r2c_impl(const Plan& p, const void* in, void* out, int n, int64_t rows, int nout, const void* fout,
                           double scale, hipStream_t st) {
  FftArgs<T> a = base_args<T>(p, n, -1);
  a.inner = 1;
  a.outer = rows;
  a.nin = n;
  a.pin = n;
  a.nout = nout;
  a.pout = nout;
  a.fac_out = (const T*)fout;
  a.scale = (T)scale;
  a.nb = lines_per_block<T>(n);
  const int64_t pairs = (rows + 1) / 2;
  const size_t lds = 2 * (size_t)n * a.nb * sizeof(cplx<T>);
  hipLaunchKernelGGL(k_fft_r2c_x<T>, dim3((unsigned)((pairs + a.nb - 1) / a.nb)), dim3(kFftThreads), lds, st,
                     (const T*)in, (cplx<T>*)out, a);
  return hipGetLastError();
}

template <typename T>
static hipError_t c2r_impl(const Plan& p, const void* in, void* out, int n, int64_t rows, int nin, const void* fin,
                           double scale, hipStream_t st) {
  FftArgs<T> a = base_args<T>(p, n, +1);
  a.inner = 1;
  a.outer = rows;
  a.nin = nin;
  a.pin = nin;
  a.nout = n;
  a.pout = n;
  a.fac_in = (const T*)fin;
  a.scale = (T)scale;
  a.nb = lines_per_block<T>(n);
  const int64_t pairs = (rows + 1) / 2;
  const size_t lds = 2 * (size_t)n * a.nb * sizeof(cplx<T>);
  hipLaunchKernelGGL(k_fft_c2r_x<T>, dim3((unsigned)((pairs + a.nb - 1) / a.nb)), dim3(kFftThreads), lds, st,
                     (const cplx<T>*)in, (T*)out, a);
  return hipGetLastError();
}

hipError_t launch_fft_r2c_x(const Plan& p, const void* in, void* out, int n, int64_t rows, int nout,
                            const void* fac_out, double scale, hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  return p.prec == FSIB_F64 ? r2c_impl<double>(p, in, out, n, rows, nout, fac_out, scale, st)
                            : r2c_impl<float>(p, in, out, n, rows, nout, fac_out, scale, st);
}

hipError_t launch_fft_c2r_x(const Plan& p, const void* in, void* out, int n, int64_t rows, int nin,
                            const void* fac_in, double scale, hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  return p.prec == FSIB_F64 ? c2r_impl<double>(p, in, out, n, rows, nin, fac_in, scale, st)
                            : c2r_impl<float>(p, in, out, n, rows, nin, fac_in, scale, st);
}

}  // namespace fsib
