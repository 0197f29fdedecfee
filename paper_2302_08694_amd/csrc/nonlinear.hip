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

// ---- length 192 = 16 x 12 in two stages ----
// The dealiasing grid of the 128^3 workload has 192 points per line.  Split as 16 x 12, each
// transform is two Stockham stages (radix 16 with no twiddles, then radix 12), and each thread keeps
// one butterfly's entries in registers, so a line crosses LDS once per direction instead of three
// times.  The kernel above spends most of its time on LDS traffic (its three radix-8/8/3 stages move
// every entry through LDS twice per stage, plus the twiddle table); this one also
//  - loads the first inverse stage's inputs straight from the half spectra (no gather in LDS),
//  - pairs the rows instead of the components in its inverse lines (line c of a row pair is
//    u_c(a) + i u_c(b)), so each product u_c1 u_c2 of both rows reads two entries, and forms the
//    products while loading the first forward stage,
//  - reads its twiddles through the vector memory path (four table entries per butterfly, which
//    stay in L1), not from LDS,
//  - unpacks the two rows of each forward line from registers, fetching the partner entry
//    Z[N - m] from the lane that holds it.
// Entries of a line sit in LDS with one pad entry per 16, so the stage-1 writes (16 apart) fall on
// distinct banks.

// e^{SG i pi j / 8} v for a compile-time j (after unrolling)
template <typename T, int SG>
__device__ __forceinline__ cplx<T> rot16(cplx<T> v, int j) {
  const T sg = (T)SG;
  const T c1 = (T)0.92387953251128675613, s1 = (T)0.38268343236508977173, h = (T)0.70710678118654752440;
  switch (j & 15) {
    case 0: return v;
    case 1: return cmul(v, mk(c1, sg * s1));
    case 2: return (v + mul_i(v, sg)) * h;
    case 3: return cmul(v, mk(s1, sg * c1));
    case 4: return mul_i(v, sg);
    case 6: return (mul_i(v, sg) - v) * h;
    case 9: return cmul(v, mk(-c1, -sg * s1));
    default: return cmul(v, mk(cos((T)3.14159265358979323846 * j / 8), sg * sin((T)3.14159265358979323846 * j / 8)));
  }
}

// In-place DFT of 16 entries, x[k] <- sum_n x[n] e^{SG 2 pi i n k / 16}: 4 x 4 Cooley-Tukey.
template <typename T, int SG>
__device__ __forceinline__ void dft16(cplx<T>* x) {
  const T sg = (T)SG;
  cplx<T> y[16];
#pragma unroll
  for (int n1 = 0; n1 < 4; ++n1) {
    cplx<T> u[4] = {x[n1], x[n1 + 4], x[n1 + 8], x[n1 + 12]};
    bfly<T, 4>(u, sg);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) y[n1 * 4 + k2] = rot16<T, SG>(u[k2], n1 * k2);
  }
#pragma unroll
  for (int k2 = 0; k2 < 4; ++k2) {
    cplx<T> u[4] = {y[k2], y[4 + k2], y[8 + k2], y[12 + k2]};
    bfly<T, 4>(u, sg);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) x[4 * k1 + k2] = u[k1];
  }
}

// In-place DFT of 12 entries (prime-factor 3 x 4, no twiddles): input n = (4 n1 + 3 n2) mod 12,
// output k = (4 k1 + 9 k2) mod 12, so that n k = 4 n1 k1 + 3 n2 k2 (mod 12).
template <typename T, int SG>
__device__ __forceinline__ void dft12(cplx<T>* x) {
  const T sg = (T)SG;
  cplx<T> y[3][4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    cplx<T> u[3] = {x[(3 * n2) % 12], x[(4 + 3 * n2) % 12], x[(8 + 3 * n2) % 12]};
    bfly<T, 3>(u, sg);
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1) y[k1][n2] = u[k1];
  }
#pragma unroll
  for (int k1 = 0; k1 < 3; ++k1) {
    cplx<T> u[4] = {y[k1][0], y[k1][1], y[k1][2], y[k1][3]};
    bfly<T, 4>(u, sg);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) x[(4 * k1 + 9 * k2) % 12] = u[k2];
  }
}

__device__ __forceinline__ constexpr int at16(int t) { return t + (t >> 4); }

// z[j] *= w^j (j = 1..11) for w = tw[r] = e^{-2 pi i r / 192}, conjugated when CONJ.  Four table
// entries are loaded (w, w^2, w^4, w^8, exact to rounding) and the others formed as products of two
// or three of them, so the eleven twiddles never sit in registers at once.
template <typename T, bool CONJ>
__device__ __forceinline__ void twiddle12(cplx<T>* z, const cplx<T>* __restrict__ tw, int r) {
  cplx<T> w1 = tw[r], w2 = tw[2 * r], w4 = tw[4 * r], w8 = tw[8 * r];
  if (CONJ) {
    w1 = conj(w1);
    w2 = conj(w2);
    w4 = conj(w4);
    w8 = conj(w8);
  }
  const cplx<T> w3 = cmul(w1, w2);
  z[1] = cmul(z[1], w1);
  z[2] = cmul(z[2], w2);
  z[3] = cmul(z[3], w3);
  z[4] = cmul(z[4], w4);
  z[5] = cmul(z[5], cmul(w1, w4));
  z[6] = cmul(z[6], cmul(w2, w4));
  z[7] = cmul(z[7], cmul(w3, w4));
  z[8] = cmul(z[8], w8);
  z[9] = cmul(z[9], cmul(w1, w8));
  z[10] = cmul(z[10], cmul(w2, w8));
  z[11] = cmul(z[11], cmul(w3, w8));
}
constexpr int kNl192Threads = 192;         // 12 lines of 16 lanes
constexpr int kNl192LineStride = 192 + 12;  // padded line in LDS

// Two row pairs per workgroup: 6 inverse lines (row pair q, component c), then 12 forward lines
// (row pair q, product f) in the same LDS buffer.  Thread (line = tid / 16, r = tid % 16).
template <typename T, int HX>
__global__ __launch_bounds__(kNl192Threads) void k_nl_xpass_16x12(const cplx<T>* __restrict__ in,
                                                                  cplx<T>* __restrict__ out,
                                                                  const cplx<T>* __restrict__ tw, int64_t rows,
                                                                  T inv_cells) {
  constexpr int N = 192, LS = kNl192LineStride;
  extern __shared__ char smem_raw[];
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
  const int tid = threadIdx.x, ln = tid >> 4, r = tid & 15;
  const int64_t pair0 = (int64_t)blockIdx.x * 2;
  const int64_t cs = rows * HX;
  // ---- inverse, stage 1 (radix 16 over t = r + 12 j), inputs from the half spectra ----
  if (ln < 6 && r < 12) {
    const int q = ln / 3, c = ln - 3 * q;
    const int64_t ra = 2 * (pair0 + q), rb = ra + 1;
    const cplx<T>* pa = ra < rows ? in + c * cs + ra * HX : nullptr;
    const cplx<T>* pb = rb < rows ? in + c * cs + rb * HX : nullptr;
    cplx<T> x[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int t = r + 12 * j;
      const bool front = 2 * t <= N;
      const int m = front ? t : N - t;
      cplx<T> A = mk((T)0, (T)0), B = mk((T)0, (T)0);
      if (m < HX) {
        if (pa) A = pa[m];
        if (pb) B = pb[m];
      }
      if (m == 0) {  // 2 m = N never holds a mode (HX <= N / 2)
        A.y = (T)0;
        B.y = (T)0;
      } else if (!front) {
        A = conj(A);
        B = conj(B);
      }
      x[j] = mk(A.x - B.y, A.y + B.x);
    }
    dft16<T, +1>(x);
    cplx<T>* L = buf + ln * LS;
#pragma unroll
    for (int j = 0; j < 16; ++j) L[at16(16 * r + j)] = x[j];
  }
  __syncthreads();
  // ---- inverse, stage 2 (radix 12 over t = r + 16 j, twiddles e^{+2 pi i j r / N}), in place ----
  if (ln < 6) {
    cplx<T> z[12];
    cplx<T>* L = buf + ln * LS;
#pragma unroll
    for (int j = 0; j < 12; ++j) z[j] = L[at16(r + 16 * j)];
    twiddle12<T, true>(z, tw, r);
    dft12<T, +1>(z);
#pragma unroll
    for (int j = 0; j < 12; ++j) L[at16(r + 16 * j)] = z[j];
  }
  __syncthreads();
  // ---- products of both rows packed as prod_f(a) + i prod_f(b), forward stage 1 (radix 16) ----
  const int q = ln / 6, f = ln - 6 * q;
  cplx<T> x[16];
  if (r < 12) {
    // product f = u_c1 u_c2 in the order xx, xy, xz, yy, yz, zz
    const int c1 = f < 3 ? 0 : (f < 5 ? 1 : 2);
    const int c2 = f < 3 ? f : (f < 5 ? f - 2 : 2);
    const cplx<T>* L1 = buf + (3 * q + c1) * LS;
    const cplx<T>* L2 = buf + (3 * q + c2) * LS;
    // squares and cross products on separate paths: a select between the two (one read for a
    // square) kept both operands of all 16 positions in registers (128 VGPRs in FP64)
    if (c1 == c2) {
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const cplx<T> v = L1[at16(r + 12 * j)];
        x[j] = mk(v.x * v.x, v.y * v.y);
      }
    } else {
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int t = at16(r + 12 * j);
        const cplx<T> v1 = L1[t], v2 = L2[t];
        x[j] = mk(v1.x * v2.x, v1.y * v2.y);
      }
    }
    dft16<T, -1>(x);
  }
  __syncthreads();  // every inverse entry has been read
  if (r < 12) {
    cplx<T>* L = buf + ln * LS;
#pragma unroll
    for (int j = 0; j < 16; ++j) L[at16(16 * r + j)] = x[j];
  }
  __syncthreads();
  // ---- forward, stage 2 (radix 12, twiddles e^{-2 pi i j r / N}) and the unpack ----
  cplx<T> z[12];
  {
    const cplx<T>* L = buf + ln * LS;
#pragma unroll
    for (int j = 0; j < 12; ++j) z[j] = L[at16(r + 16 * j)];
    twiddle12<T, false>(z, tw, r);
    dft12<T, -1>(z);
  }
  // This thread holds Z[r + 16 j].  Modes m = r + 16 s < HX (s <= 3, and s = 4 for r = 0) need
  // Z[N - m]: for r > 0 that is Z[(16 - r) + 16 (11 - s)] of lane 16 - r of the same line, for r = 0
  // it is this thread's Z[16 ((12 - s) mod 12)].
  const int partner = (threadIdx.x & 63 & ~15) | ((16 - r) & 15);
  const int64_t ra = 2 * (pair0 + q), rb = ra + 1;
  const T sc = (T)0.5 * inv_cells;
  cplx<T>* oa = out + f * cs + ra * HX;
  cplx<T>* ob = out + f * cs + rb * HX;
#pragma unroll
  for (int s = 0; s < 5; ++s) {
    cplx<T> zc;
    if (s < 4) {
      zc.x = __shfl(z[11 - s].x, partner, 64);
      zc.y = __shfl(z[11 - s].y, partner, 64);
      if (r == 0) zc = z[(12 - s) % 12];
    } else {
      zc = z[8];
    }
    const int m = r + 16 * s;
    if ((s < 4 || r == 0) && m < HX && ra < rows) {
      zc = conj(zc);
      const cplx<T> su = z[s] + zc, d = z[s] - zc;
      oa[m] = su * sc;
      if (rb < rows) ob[m] = mk(d.y * sc, -d.x * sc);
    }
  }
}

template <typename T>
static hipError_t nl_impl(const Plan& p, const void* in, void* out, int stages, hipStream_t st) {
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
  // two or three FFT stages on 192-point lines (the caller's choice)
  if (p.dim == 3 && n == 192 && pp == 2 && p.Hx == 65 && stages == 2)
    hipLaunchKernelGGL((k_nl_xpass_16x12<T, 65>), dim3(nblk), dim3(kNl192Threads),
                       (size_t)12 * kNl192LineStride * sizeof(cplx<T>), st, (const cplx<T>*)in, (cplx<T>*)out, a.tw,
                       rows, inv);
  else if (p.dim == 3 && n == 192 && pp == 2 && p.Hx == 65)
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

hipError_t launch_nl_xpass(const Plan& p, const void* in, void* out, int stages, hipStream_t st) {
  return p.prec == FSIB_F64 ? nl_impl<double>(p, in, out, stages, st) : nl_impl<float>(p, in, out, stages, st);
}

}  // namespace fsib
