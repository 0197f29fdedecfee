// Dealiased quadratic products of the velocity along x in one kernel (three-halves rule, Sec. 3.1).
//
// Input: the velocity components on the dealiasing grid in y and z, still as half spectra in x
// ([d][rows][Hx] complex, rows = Ntilde_z * Ntilde_y).  For a pair of rows (a, b) a workgroup
// forms the complex lines u_x(a) + i u_y(a), u_x(b) + i u_y(b) (and u_z(a) + i u_z(b) in 3D),
// inverse-transforms them in LDS (length Ntilde_x), multiplies u_alpha u_beta point by point, packs
// the products of the two rows into complex lines, forward-transforms them and keeps the first Hx
// modes of each -- so neither the velocity nor the products on the padded grid ever reach memory.
// Output: the products' half spectra in x ([nprod][rows][Hx]), scaled by 1/Ntilde^d (the H of
// eq. nonlinear_physical), ready for the forward passes along y and z.
#include "fft_device.hpp"
#include "plan.hpp"

namespace fsib {

// N > 0: length N and PP row pairs per workgroup known at compile time; N = 0: from the arguments.
// HX > 0: the half-spectrum length known at compile time too (index divisions become multiplies and
// the gather and store loops get fixed trip counts).
template <typename T, int DIM, int N = 0, int PP = 0, int HX = 0>
__global__ __launch_bounds__(1024) void k_nl_xpass(const cplx<T>* __restrict__ in, cplx<T>* __restrict__ out,
                                                   FftArgs<T> a, int64_t rows, int hx_arg, int pp_arg, T inv_cells) {
  constexpr int IL = DIM == 3 ? 3 : 2;  // inverse lines per row pair
  constexpr int FL = DIM == 3 ? 6 : 3;  // forward lines per row pair (products)
  constexpr int NTHR = (FL * PP * N + kEPT - 1) / kEPT;
  // loads per thread in the gather: all kEPT slots unless the sizes are compile-time
  constexpr int GJ = N > 0 ? (IL * PP * N + NTHR - 1) / NTHR : kEPT;
  extern __shared__ char smem_raw[];
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
  const int n = N > 0 ? N : a.n, nthr = N > 0 ? NTHR : (int)blockDim.x, pp = N > 0 ? PP : pp_arg;
  const int hx = HX > 0 ? HX : hx_arg;
  cplx<T>* twl = buf + lpad_len(FL * pp * n);  // lines padded (lpad)
  const int64_t pair0 = (int64_t)blockIdx.x * pp;
  const int64_t cs = rows * hx;  // component stride of in/out
  // ---- gather the Hermitian-extended lines (inverse) ----
  const int nin = IL * pp * n;
  // With every size fixed at compile time and the threads dividing into the lines, each thread owns
  // JP positions t = tl + TPL j of one line: its line's component, rows and base pointers are worked
  // out once, and consecutive threads read consecutive modes.
  constexpr bool LINE_MAP = N > 0 && HX > 0 && NTHR % (IL * PP) == 0 && N % (NTHR / (IL * PP > 0 ? IL * PP : 1)) == 0;
  if constexpr (LINE_MAP) {
    constexpr int TPL = NTHR / (IL * PP), JP = N / TPL;
    const int ln = threadIdx.x / TPL, tl = threadIdx.x - ln * TPL;
    const int q = ln / IL, l = ln - q * IL;
    const int64_t ra = 2 * (pair0 + q), rb = ra + 1;
    // line l: (comp, row) of its real part A and imaginary part B
    const int ca = l == 2 ? 2 : 0, cb = l == 2 ? 2 : 1;
    const int64_t rowa = l == 1 ? rb : ra, rowb = l == 0 ? ra : rb;
    const cplx<T>* pa = rowa < rows ? in + ca * cs + rowa * HX : nullptr;
    const cplx<T>* pb = rowb < rows ? in + cb * cs + rowb * HX : nullptr;
    cplx<T> A[JP], B[JP];
#pragma unroll
    for (int j = 0; j < JP; ++j) {
      const int t = tl + TPL * j;
      const int m = 2 * t <= N ? t : N - t;
      A[j] = mk((T)0, (T)0);
      B[j] = mk((T)0, (T)0);
      if (m < HX) {
        if (pa) A[j] = pa[m];
        if (pb) B[j] = pb[m];
      }
    }
    stage_twiddles(a.tw, twl, N);  // behind the data loads, so both latencies overlap
#pragma unroll
    for (int j = 0; j < JP; ++j) {
      const int t = tl + TPL * j;
      const bool front = 2 * t <= N;
      const int m = front ? t : N - t;
      cplx<T> x = A[j], y = B[j];
      if (m == 0 || 2 * m == N) {
        x.y = (T)0;
        y.y = (T)0;
      } else if (!front) {
        x = conj(x);
        y = conj(y);
      }
      buf[lpad(ln * N + t)] = mk(x.x - y.y, x.y + y.x);
    }
  } else {
  cplx<T> A[GJ], B[GJ];
#pragma unroll
  for (int j = 0; j < GJ; ++j) {
    const int e = threadIdx.x + j * nthr;
    A[j] = mk((T)0, (T)0);
    B[j] = mk((T)0, (T)0);
    if (e < nin) {
      const int ln = e / n, t = e - ln * n;
      const int q = ln / IL, l = ln - q * IL;
      const int64_t ra = 2 * (pair0 + q), rb = ra + 1;
      const int m = 2 * t <= n ? t : n - t;
      if (m < hx) {
        // line l: (comp, row) of its real part A and imaginary part B
        int ca, cb;
        int64_t rowa, rowb;
        if (l == 0) {
          ca = 0; cb = 1; rowa = ra; rowb = ra;
        } else if (l == 1) {
          ca = 0; cb = 1; rowa = rb; rowb = rb;
        } else {
          ca = 2; cb = 2; rowa = ra; rowb = rb;
        }
        if (rowa < rows) A[j] = in[ca * cs + rowa * hx + m];
        if (rowb < rows) B[j] = in[cb * cs + rowb * hx + m];
      }
    }
  }
  stage_twiddles(a.tw, twl, n);  // behind the data loads, so both latencies overlap
#pragma unroll
  for (int j = 0; j < GJ; ++j) {
    const int e = threadIdx.x + j * nthr;
    if (e < nin) {
      const int t = e % n;
      const bool front = 2 * t <= n;
      const int m = front ? t : n - t;
      cplx<T> x = A[j], y = B[j];
      if (m == 0 || 2 * m == n) {
        x.y = (T)0;
        y.y = (T)0;
      } else if (!front) {
        x = conj(x);
        y = conj(y);
      }
      buf[lpad(e)] = mk(x.x - y.y, x.y + y.x);
    }
  }
  }
  __syncthreads();
  if constexpr (N > 0)
    stockham_ct_dir<T, true, N, IL * PP, NTHR, +1>(buf, twl);
  else
    stockham<T, true>(a, buf, twl, IL * pp, +1);
  // ---- products, packed two rows per complex line: line (q, f) = prod_f(row a) + i prod_f(row b) ----
  constexpr int PPT = (kEPT + FL - 1) / FL;  // (pair, t) positions per thread
  T pa[PPT][FL], pb[PPT][FL];
  int pos[PPT];
#pragma unroll
  for (int j = 0; j < PPT; ++j) {
    const int e = threadIdx.x + j * nthr;
    pos[j] = -1;
    if (e < pp * n) {
      const int q = e / n, t = e - q * n;
      pos[j] = e;
      const cplx<T> l0 = buf[lpad((q * IL + 0) * n + t)], l1 = buf[lpad((q * IL + 1) * n + t)];
      const T uxa = l0.x, uya = l0.y, uxb = l1.x, uyb = l1.y;
      if constexpr (DIM == 3) {
        const cplx<T> l2 = buf[lpad((q * IL + 2) * n + t)];
        const T uza = l2.x, uzb = l2.y;
        pa[j][0] = uxa * uxa; pa[j][1] = uxa * uya; pa[j][2] = uxa * uza;
        pa[j][3] = uya * uya; pa[j][4] = uya * uza; pa[j][5] = uza * uza;
        pb[j][0] = uxb * uxb; pb[j][1] = uxb * uyb; pb[j][2] = uxb * uzb;
        pb[j][3] = uyb * uyb; pb[j][4] = uyb * uzb; pb[j][5] = uzb * uzb;
      } else {
        pa[j][0] = uxa * uxa; pa[j][1] = uxa * uya; pa[j][2] = uya * uya;
        pb[j][0] = uxb * uxb; pb[j][1] = uxb * uyb; pb[j][2] = uyb * uyb;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < PPT; ++j) {
    if (pos[j] >= 0) {
      const int q = pos[j] / n, t = pos[j] - q * n;
#pragma unroll
      for (int f = 0; f < FL; ++f) buf[lpad((q * FL + f) * n + t)] = mk(pa[j][f], pb[j][f]);
    }
  }
  __syncthreads();
  if constexpr (N > 0)
    stockham_ct_dir<T, true, N, FL * PP, NTHR, -1>(buf, twl);
  else
    stockham<T, true>(a, buf, twl, FL * pp, -1);
  // ---- unpack the two rows of each line, keep m < Hx ----
  constexpr bool STORE_MAP = N > 0 && HX > 0 && NTHR % (FL * PP > 0 ? FL * PP : 1) == 0;
  if constexpr (STORE_MAP) {
    // each thread owns modes m = ml + TPS j of one line (consecutive threads, consecutive modes)
    constexpr int TPS = NTHR / (FL * PP), JS = (HX + TPS - 1) / TPS;
    const int ln = threadIdx.x / TPS, ml = threadIdx.x - ln * TPS;
    const int q = ln / FL, f = ln - q * FL;
    const int64_t ra = 2 * (pair0 + q), rb = ra + 1;
    if (ra < rows) {
      cplx<T>* oa = out + f * cs + ra * HX;
      cplx<T>* ob = out + f * cs + rb * HX;
      const bool hasb = rb < rows;
      const T sc = (T)0.5 * inv_cells;
#pragma unroll
      for (int j = 0; j < JS; ++j) {
        const int m = ml + TPS * j;
        if (m < HX) {
          const cplx<T> Z = buf[lpad(ln * N + m)];
          const cplx<T> Zc = conj(buf[lpad(ln * N + (m == 0 ? 0 : N - m))]);
          const cplx<T> su = Z + Zc, d = Z - Zc;
          oa[m] = su * sc;
          if (hasb) ob[m] = mk(d.y * sc, -d.x * sc);
        }
      }
    }
    return;
  }
  const int nst = FL * pp * hx;
  constexpr int SJ = HX > 0 ? (FL * PP * HX + NTHR - 1) / NTHR : 1;  // compile-time trip count
#pragma unroll
  for (int j = 0; j < (HX > 0 ? SJ : 1); ++j)
  for (int e = threadIdx.x + j * nthr; e < nst; e += (HX > 0 ? nst : nthr)) {
    const int ln = e / hx, m = e - ln * hx;
    const int q = ln / FL, f = ln - q * FL;
    const int64_t ra = 2 * (pair0 + q), rb = ra + 1;
    if (ra >= rows) continue;
    const cplx<T> Z = buf[lpad(ln * n + m)];
    const cplx<T> Zc = conj(buf[lpad(ln * n + (m == 0 ? 0 : n - m))]);
    const T s = (T)0.5 * inv_cells;
    const cplx<T> su = Z + Zc, d = Z - Zc;
    out[f * cs + ra * hx + m] = su * s;
    if (rb < rows) out[f * cs + rb * hx + m] = mk(d.y * s, -d.x * s);
  }
}

template <typename T>
static hipError_t nl_impl(const Plan& p, const void* in, void* out, hipStream_t st) {
  const int n = (int)p.nd[0];
  FftArgs<T> a;
  const PassMasks none;
  a.line = none.line;
  a.ld = none.ld;
  a.st = none.st;
  a.rows = none.rows;
  a.n = n;
  a.nst = radix_plan(n, a.radix);
  a.tw = (const cplx<T>*)p.tw.at(n);
  a.sign = -1;
  a.inner = 1;
  a.outer = 0;
  a.nin = a.pin = a.nout = a.pout = n;
  a.fac_in = a.fac_out = nullptr;
  a.scale = (T)1;
  a.nb = 0;
  const int64_t rows = p.dim == 3 ? p.nd[2] * p.nd[1] : p.nd[1];
  const int fl = p.dim == 3 ? 6 : 3;
  // row pairs per workgroup: the forward lines fit 2304 complex entries (36 KiB in FP64) and 1024
  // threads
  int pp = (int)(2304 / ((size_t)fl * n));
  if (pp < 1) pp = 1;
  while (pp > 1 && (fl * pp * n + kEPT - 1) / kEPT > 1024) --pp;
  const int64_t pairs = (rows + 1) / 2;
  if (pp > pairs) pp = (int)pairs;
  const int nthr = (fl * pp * n + kEPT - 1) / kEPT;
  const size_t lds = (size_t)(lpad_len(fl * pp * n) + n) * sizeof(cplx<T>);
  const unsigned nblk = (unsigned)((pairs + pp - 1) / pp);
  const T inv = (T)(1.0 / (double)p.dealias_cells());
  const bool prof = prof_on(p, PROF_NL_X);
  if (prof) prof_start(p, st);
  if (p.dim == 3 && n == 192 && pp == 2 && p.Hx == 65)
    hipLaunchKernelGGL((k_nl_xpass<T, 3, 192, 2, 65>), dim3(nblk), dim3(nthr), lds, st, (const cplx<T>*)in,
                       (cplx<T>*)out, a, rows, (int)p.Hx, pp, inv);
  else if (p.dim == 3 && n == 192 && pp == 2)
    hipLaunchKernelGGL((k_nl_xpass<T, 3, 192, 2>), dim3(nblk), dim3(nthr), lds, st, (const cplx<T>*)in, (cplx<T>*)out,
                       a, rows, (int)p.Hx, pp, inv);
  else if (p.dim == 3 && n == 96 && pp == 4)
    hipLaunchKernelGGL((k_nl_xpass<T, 3, 96, 4>), dim3(nblk), dim3(nthr), lds, st, (const cplx<T>*)in, (cplx<T>*)out,
                       a, rows, (int)p.Hx, pp, inv);
  else if (p.dim == 3 && n == 384 && pp == 1)
    hipLaunchKernelGGL((k_nl_xpass<T, 3, 384, 1>), dim3(nblk), dim3(nthr), lds, st, (const cplx<T>*)in, (cplx<T>*)out,
                       a, rows, (int)p.Hx, pp, inv);
  else if (p.dim == 3)
    hipLaunchKernelGGL((k_nl_xpass<T, 3>), dim3(nblk), dim3(nthr), lds, st, (const cplx<T>*)in, (cplx<T>*)out, a, rows,
                       (int)p.Hx, pp, inv);
  else
    hipLaunchKernelGGL((k_nl_xpass<T, 2>), dim3(nblk), dim3(nthr), lds, st, (const cplx<T>*)in, (cplx<T>*)out, a, rows,
                       (int)p.Hx, pp, inv);
  // algorithmic bytes: dim velocity half-spectrum rows in, nprod product rows out
  if (prof) prof_stop(p, (double)(p.dim + p.nprod()) * rows * p.Hx * sizeof(cplx<T>), st);
  return hipGetLastError();
}

// The x pass of the dealiased product holds the forward lines of one row pair (3 in 2D, 6 in 3D)
// in one workgroup of at most 1024 threads.
bool nl_line_fits(const Plan& p, int n) {
  const int fl = p.dim == 3 ? 6 : 3;
  if ((fl * n + kEPT - 1) / kEPT > 1024) return false;
  const size_t cs = p.prec == FSIB_F64 ? sizeof(cplx<double>) : sizeof(cplx<float>);
  return (size_t)(lpad_len(fl * n) + n) * cs <= (size_t)p.lds_max;
}

hipError_t launch_nl_xpass(const Plan& p, const void* in, void* out, hipStream_t st) {
  return p.prec == FSIB_F64 ? nl_impl<double>(p, in, out, st) : nl_impl<float>(p, in, out, st);
}

}  // namespace fsib
