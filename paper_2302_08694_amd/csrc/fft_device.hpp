// Device building blocks of the LDS Stockham FFT (shared by the FFT passes and the fused kernels).
//
// Stockham stage (radix r, p = product of the radices already applied, m = n/r): butterfly i < m,
// k = i mod p, inputs x[i + q m] (q < r) twiddled by exp(sign 2 pi i q k / (p r)), outputs
// y[(i - k) r + k + q p].  Each thread reads its butterfly inputs into registers, the workgroup
// synchronises, and the outputs are written back into the same LDS buffer.  The twiddle table
// exp(-2 pi i t / n) is staged in LDS once per workgroup.
#pragma once

#include "common.hpp"

namespace fsib {

constexpr int kEPT = 8;            // complex elements per thread
constexpr int kMaxFftThreads = 512;

template <typename T, int R>
__device__ __forceinline__ void bfly(cplx<T>* u, T sg) {
  if constexpr (R == 2) {
    const cplx<T> a = u[0], b = u[1];
    u[0] = a + b;
    u[1] = a - b;
  } else if constexpr (R == 4) {
    const cplx<T> s02 = u[0] + u[2], d02 = u[0] - u[2], s13 = u[1] + u[3], d13 = u[1] - u[3];
    u[0] = s02 + s13;
    u[2] = s02 - s13;
    u[1] = d02 + mul_i(d13, sg);
    u[3] = d02 - mul_i(d13, sg);
  } else if constexpr (R == 8) {
    // two length-4 transforms of the even and odd samples, combined with exp(sign i pi k / 4)
    cplx<T> e[4] = {u[0], u[2], u[4], u[6]};
    cplx<T> o[4] = {u[1], u[3], u[5], u[7]};
    bfly<T, 4>(e, sg);
    bfly<T, 4>(o, sg);
    const T c = (T)0.70710678118654752440;
    const cplx<T> o1 = (o[1] + mul_i(o[1], sg)) * c;
    const cplx<T> o2 = mul_i(o[2], sg);
    const cplx<T> o3 = (mul_i(o[3], sg) - o[3]) * c;
    u[0] = e[0] + o[0];
    u[4] = e[0] - o[0];
    u[1] = e[1] + o1;
    u[5] = e[1] - o1;
    u[2] = e[2] + o2;
    u[6] = e[2] - o2;
    u[3] = e[3] + o3;
    u[7] = e[3] - o3;
  } else if constexpr (R == 3) {
    const T c = (T)-0.5, s = (T)0.86602540378443864676;
    const cplx<T> t = u[1] + u[2], d = u[1] - u[2];
    const cplx<T> a = u[0] + t * c;
    u[0] = u[0] + t;
    const cplx<T> b = mul_i(d, sg * s);
    u[1] = a + b;
    u[2] = a - b;
  } else {  // R == 5
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

// Contiguous lines in LDS are padded by one entry per 8: a Stockham stage writes its outputs R
// entries apart, and unpadded the lanes of a wavefront would hit the same few banks (measured
// bank-conflict cycles above the kernel's busy cycles in the fused nonlinear pass).
__host__ __device__ constexpr int lpad(int x) { return x + (x >> 3); }
__host__ __device__ constexpr int lpad_len(int m) { return m + (m >> 3) + 1; }  // entries for m lines' worth

// LDS index of entry t of line b: lines contiguous and padded (x passes) or interleaved (strided
// passes, whose lanes already write whole 128-byte runs).
template <bool CONTIG>
__device__ __forceinline__ int lidx(int t, int b, int n, int nb) {
  return CONTIG ? lpad(b * n + t) : t * nb + b;
}

// Copies the n twiddles into LDS (caller synchronises before the first stage).
template <typename T>
__device__ __forceinline__ void stage_twiddles(const cplx<T>* __restrict__ tw, cplx<T>* twl, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) twl[i] = tw[i];
}

template <typename T, bool CONTIG, int R>
__device__ __forceinline__ void stage(int n, cplx<T>* buf, const cplx<T>* twl, int p, int nb, int sign) {
  constexpr int NBF = (kEPT + R - 1) / R;
  const int m = n / R;
  const int total = m * nb;
  const int nthr = blockDim.x;
  const int twstride = n / (p * R);
  const T sg = (T)sign;
  cplx<T> u[NBF][R];
  int ii[NBF], bb[NBF];
#pragma unroll
  for (int j = 0; j < NBF; ++j) {
    const int bf = threadIdx.x + j * nthr;
    ii[j] = -1;
    bb[j] = 0;
    if (bf < total) {
      int i, b;
      if (CONTIG) {
        b = bf / m;
        i = bf - b * m;
      } else {
        i = bf / nb;
        b = bf - i * nb;
      }
      ii[j] = i;
      bb[j] = b;
#pragma unroll
      for (int q = 0; q < R; ++q) u[j][q] = buf[lidx<CONTIG>(i + q * m, b, n, nb)];
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < NBF; ++j) {
    const int i = ii[j];
    if (i >= 0) {
      const int b = bb[j];
      const int k = i % p;
      if (p > 1) {
#pragma unroll
        for (int q = 1; q < R; ++q) {
          cplx<T> w = twl[q * k * twstride];
          if (sign > 0) w.y = -w.y;
          u[j][q] = cmul(u[j][q], w);
        }
      }
      bfly<T, R>(u[j], sg);
      const int j0 = (i - k) * R + k;
#pragma unroll
      for (int q = 0; q < R; ++q) buf[lidx<CONTIG>(j0 + q * p, b, n, nb)] = u[j][q];
    }
  }
  __syncthreads();
}

// All stages of nb lines of length a.n held in buf; needs blockDim.x * kEPT >= a.n * nb and the
// twiddles staged in twl.
template <typename T, bool CONTIG>
__device__ __forceinline__ void stockham(const FftArgs<T>& a, cplx<T>* buf, const cplx<T>* twl, int nb, int sign) {
  int p = 1;
  for (int s = 0; s < a.nst; ++s) {
    const int r = a.radix[s];
    if (r == 8)
      stage<T, CONTIG, 8>(a.n, buf, twl, p, nb, sign);
    else if (r == 4)
      stage<T, CONTIG, 4>(a.n, buf, twl, p, nb, sign);
    else if (r == 2)
      stage<T, CONTIG, 2>(a.n, buf, twl, p, nb, sign);
    else if (r == 3)
      stage<T, CONTIG, 3>(a.n, buf, twl, p, nb, sign);
    else
      stage<T, CONTIG, 5>(a.n, buf, twl, p, nb, sign);
    p *= r;
  }
}

// ---- the same stages with the length and the line count known at compile time ----
// For the lengths of the hot passes the index arithmetic of every stage (divisions by the line
// count, the butterfly count and the twiddle stride) folds into shifts and constant multiplies.
// The radix order is the host's (8s, then 4, 2, 3, 5).
constexpr int kCtRadices[5] = {8, 4, 2, 3, 5};
constexpr int ct_nstages(int n) {
  int m = n, k = 0;
  for (int r = 0; r < 5; ++r)
    while (m % kCtRadices[r] == 0) {
      m /= kCtRadices[r];
      ++k;
    }
  return m == 1 ? k : -1;
}
constexpr int ct_radix_at(int n, int s) {
  int m = n, k = 0;
  for (int r = 0; r < 5; ++r)
    while (m % kCtRadices[r] == 0) {
      if (k == s) return kCtRadices[r];
      m /= kCtRadices[r];
      ++k;
    }
  return 1;
}
constexpr int ct_p_before(int n, int s) {
  int p = 1;
  for (int t = 0; t < s; ++t) p *= ct_radix_at(n, t);
  return p;
}

// NTHR = blockDim.x (N * NB / kEPT for the passes; the fused nonlinear kernel runs fewer lines
// than threads in its inverse half).  SIGN = +1 or -1 fixes the transform direction at compile time
// (the products by +-1 in the butterflies and the conjugation of the twiddles fold away); SIGN = 0
// takes it from `sign` (one code path for both directions).  In the padded contiguous
// layout lpad(x + y) = lpad(x) + lpad(y) when y is a multiple of 8, so a butterfly whose stride (M
// for its inputs, P for its outputs) is a multiple of 8 computes one padded index and reaches the
// others by constant offsets.
template <typename T, bool CONTIG, int N, int NB, int NTHR, int R, int P, int SIGN>
__device__ __forceinline__ void stage_ct(cplx<T>* buf, const cplx<T>* twl, int sign) {
  constexpr int M = N / R;
  constexpr int TOTAL = M * NB;
  constexpr int NBF = (TOTAL + NTHR - 1) / NTHR;
  constexpr int TWS = N / (P * R);
  const T sg = SIGN != 0 ? (T)SIGN : (T)sign;
  cplx<T> u[NBF][R];
  int ii[NBF], bb[NBF];
#pragma unroll
  for (int j = 0; j < NBF; ++j) {
    const int bf = threadIdx.x + j * NTHR;
    ii[j] = -1;
    bb[j] = 0;
    if (TOTAL % NTHR == 0 || bf < TOTAL) {
      int i, b;
      if (CONTIG) {
        b = bf / M;
        i = bf - b * M;
      } else {
        i = bf / NB;
        b = bf - i * NB;
      }
      ii[j] = i;
      bb[j] = b;
      if constexpr (CONTIG && M % 8 == 0) {
        const int base = lpad(b * N + i);
#pragma unroll
        for (int q = 0; q < R; ++q) u[j][q] = buf[base + q * lpad(M)];
      } else {
#pragma unroll
        for (int q = 0; q < R; ++q) u[j][q] = buf[lidx<CONTIG>(i + q * M, b, N, NB)];
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < NBF; ++j) {
    const int i = ii[j];
    if (TOTAL % NTHR == 0 || i >= 0) {
      const int b = bb[j];
      const int k = i % P;
      if (P > 1) {
#pragma unroll
        for (int q = 1; q < R; ++q) {
          cplx<T> w = twl[q * k * TWS];
          if (SIGN > 0 || (SIGN == 0 && sign > 0)) w.y = -w.y;
          u[j][q] = cmul(u[j][q], w);
        }
      }
      bfly<T, R>(u[j], sg);
      const int j0 = (i - k) * R + k;
      if constexpr (CONTIG && P % 8 == 0) {
        const int base = lpad(b * N + j0);
#pragma unroll
        for (int q = 0; q < R; ++q) buf[base + q * lpad(P)] = u[j][q];
      } else {
#pragma unroll
        for (int q = 0; q < R; ++q) buf[lidx<CONTIG>(j0 + q * P, b, N, NB)] = u[j][q];
      }
    }
  }
  __syncthreads();
}

template <typename T, bool CONTIG, int N, int NB, int NTHR, int SIGN, int S = 0>
__device__ __forceinline__ void stockham_ct_dir(cplx<T>* buf, const cplx<T>* twl, int sign = SIGN) {
  if constexpr (S < ct_nstages(N)) {
    stage_ct<T, CONTIG, N, NB, NTHR, ct_radix_at(N, S), ct_p_before(N, S), SIGN>(buf, twl, sign);
    stockham_ct_dir<T, CONTIG, N, NB, NTHR, SIGN, S + 1>(buf, twl, sign);
  }
}

// Middle Stockham stages s = S .. SL-1 of a compile-time strided pass (each reads LDS, synchronises,
// writes LDS and synchronises).
template <typename T, int N, int NB, int NTHR, int S, int SL>
__device__ __forceinline__ void middle_stages(cplx<T>* buf, const cplx<T>* twl, int sign) {
  if constexpr (S < SL) {
    stage_ct<T, false, N, NB, NTHR, ct_radix_at(N, S), ct_p_before(N, S), 0>(buf, twl, sign);
    middle_stages<T, N, NB, NTHR, S + 1, SL>(buf, twl, sign);
  }
}

// Direction known only at run time (a single code path serves both; two unrolled copies measured
// no faster).
template <typename T, bool CONTIG, int N, int NB, int NTHR = N * NB / kEPT>
__device__ __forceinline__ void stockham_ct(cplx<T>* buf, const cplx<T>* twl, int sign) {
  stockham_ct_dir<T, CONTIG, N, NB, NTHR, 0>(buf, twl, sign);
}

}  // namespace fsib
