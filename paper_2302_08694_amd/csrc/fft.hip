// Batched mixed-radix (2, 3, 4, 5) Stockham FFT passes in LDS.
//
// One pass transforms every line of one axis of a [outer][len][inner] complex array.  A
// workgroup holds `nb` lines in one LDS buffer (contiguous lines for the x axis; `nb` neighbouring
// columns for strided axes, so that global accesses stay coalesced).  Each thread owns kEPT
// elements: the load phase issues all of its global loads before writing LDS, and every Stockham
// stage reads its butterfly inputs into registers, synchronises, and writes the outputs back into
// the same buffer.  Zero padding of the input, truncation of the output to a mode set in FFT order,
// and per-mode real factors (the NUFFT deconvolution, App. A eqs. type1_deco and type2_divi) are
// folded into the load and store, so pruned transforms read and write only entries that exist.
// Real-data passes along x pack two real lines into one complex line.
//
// Stockham stage (radix r, p = product of the radices already applied, m = n/r): butterfly i < m,
// k = i mod p, inputs x[i + q m] (q < r) twiddled by exp(sign 2 pi i q k / (p r)), outputs
// y[(i - k) r + k + q p].
#include "fft_device.hpp"
#include "plan.hpp"

namespace fsib {

// Occupancy flags live in dynamic LDS after the lines and the twiddles: one byte per line of the
// workgroup (x passes: 2 per pair) or per loaded entry (strided passes).
template <typename T>
__device__ __forceinline__ uint8_t* flag_area(cplx<T>* twl, int n) {
  return reinterpret_cast<uint8_t*>(twl + n);
}
static size_t flag_bytes(int nflags) { return (size_t)((nflags + 15) / 16 * 16); }
// workgroup size of the passes: 2048 complex entries in LDS (256 threads of kEPT entries) in both
// precisions (measured at 128^3: 1024 or 4096 entries are slower in FP64, 4096 is slower in FP32)
constexpr int kFftWgEntries = 2048;

// Strided pass with the length and the line count known at compile time, its first and last Stockham
// stages in registers: the first stage's butterflies read their inputs straight from memory (zero
// padding and the per-entry factors folded in) and write the outputs to LDS; the middle stages run in
// LDS; the last stage reads LDS and stores its outputs straight to memory (truncation, factors and
// the store mask folded in).  Against staging the whole line in LDS this halves the LDS traffic and
// drops four workgroup barriers.  Thread bf of a stage owns butterfly i = bf / NB of column
// b = bf % NB, so the lanes of a wavefront read and write runs of NB adjacent columns.
template <typename T, int N, int NB>
__device__ __forceinline__ void c2c_strided_ct(const cplx<T>* __restrict__ in, cplx<T>* __restrict__ out,
                                               const FftArgs<T>& a, Blk wb) {
  constexpr int NTHR = N * NB / kEPT;
  constexpr int NS = ct_nstages(N);
  static_assert(NS >= 2, "two stages at least");
  extern __shared__ char smem_raw[];
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* twl = buf + N * NB;
  uint8_t* fld = flag_area(twl, N);
  // plain numbering only where whole lines may be skipped (a line mask): per-entry masks leave
  // every workgroup some work, so neighbours stay on one XCD
  const int64_t lin0 = wb.x + wb.y * wb.nx;
  const int64_t lin = a.line.m ? lin0 : xcd_linear(lin0, wb.nx * wb.ny);
  const int64_t q0 = (lin % wb.nx) * NB;
  const int64_t o0 = lin / wb.nx;
  const int ncol = (int)(a.inner - q0 < NB ? a.inner - q0 : NB);
  const bool line = !a.line.m || a.line.m[mask_index(a.line, o0, 0)];
  for (int i = threadIdx.x; i < a.nin; i += NTHR) fld[i] = line && (!a.ld.m || a.ld.m[mask_index(a.ld, o0, i)]);
  if (!__syncthreads_or(line)) return;
  const int sign = a.sign;
  const T sg = (T)sign;
  constexpr int RL = ct_radix_at(N, NS - 1);
  constexpr int PL = ct_p_before(N, NS - 1);
  constexpr int ML = N / RL;
  constexpr int TOTL = ML * NB;
  constexpr int NBFL = (TOTL + NTHR - 1) / NTHR;
  static_assert(NBFL * RL <= 64, "store flags fit 64 bits");
  // store flags of this thread's outputs (bit j * RL + q), fetched before the stages so their
  // latency overlaps the data loads
  const int pout = a.pout, hiout = N - (a.nout - a.pout);  // outputs t in [pout, hiout) are dropped
  uint64_t keep = 0;
#pragma unroll
  for (int j = 0; j < NBFL; ++j) {
    const int bf = threadIdx.x + j * NTHR;
    if (!(TOTL % NTHR == 0 || bf < TOTL)) continue;
    const int i = bf / NB, b = bf - (bf / NB) * NB;
    const int k = i % PL, j0 = (i - k) * RL + k;
#pragma unroll
    for (int q = 0; q < RL; ++q) {
      const int t = j0 + q * PL;
      const int io = t < pout ? t : (t >= hiout ? t - (N - a.nout) : -1);
      const bool kp = io >= 0 && b < ncol && (!a.st.m || a.st.m[mask_index(a.st, o0, io)] != 0);
      if (kp) keep |= 1ull << (j * RL + q);
    }
  }
  // ---- first stage (radix R0, no twiddles) from memory ----
  {
    constexpr int R0 = ct_radix_at(N, 0);
    constexpr int M0 = N / R0;
    constexpr int TOT = M0 * NB;
    constexpr int NBF = (TOT + NTHR - 1) / NTHR;
    const int pin = a.pin, hi = N - (a.nin - a.pin);  // entries t in [pin, hi) are the zero padding
    cplx<T> u[NBF][R0];
#pragma unroll
    for (int j = 0; j < NBF; ++j) {
      const int bf = threadIdx.x + j * NTHR;
      const bool valid = TOT % NTHR == 0 || bf < TOT;
      const int i = bf / NB, b = bf - (bf / NB) * NB;
#pragma unroll
      for (int q = 0; q < R0; ++q) {
        const int t = i + q * M0;
        const int ie = t < pin ? t : (t >= hi ? t - (N - a.nin) : -1);
        u[j][q] = mk((T)0, (T)0);
        if (valid && ie >= 0 && b < ncol && fld[ie]) {
          cplx<T> v = in[(o0 * a.nin + ie) * a.inner + q0 + b];
          if (a.fac_in) v = v * a.fac_in[ie];
          u[j][q] = v;
        }
      }
    }
    stage_twiddles(a.tw, twl, N);  // behind the data loads
#pragma unroll
    for (int j = 0; j < NBF; ++j) {
      const int bf = threadIdx.x + j * NTHR;
      if (TOT % NTHR == 0 || bf < TOT) {
        const int i = bf / NB, b = bf - (bf / NB) * NB;
        bfly<T, R0>(u[j], sg);
#pragma unroll
        for (int q = 0; q < R0; ++q) buf[(i * R0 + q) * NB + b] = u[j][q];
      }
    }
    __syncthreads();
  }
  middle_stages<T, N, NB, NTHR, 1, NS - 1>(buf, twl, sign);
  // ---- last stage from LDS to memory ----
  {
    constexpr int TWS = N / (PL * RL);
#pragma unroll
    for (int j = 0; j < NBFL; ++j) {
      const int bf = threadIdx.x + j * NTHR;
      if (!(TOTL % NTHR == 0 || bf < TOTL)) continue;
      if (((keep >> (j * RL)) & ((1ull << RL) - 1)) == 0) continue;  // nothing of this butterfly is stored
      const int i = bf / NB, b = bf - (bf / NB) * NB;
      cplx<T> u[RL];
#pragma unroll
      for (int q = 0; q < RL; ++q) u[q] = buf[(i + q * ML) * NB + b];
      const int k = i % PL;
#pragma unroll
      for (int q = 1; q < RL; ++q) {
        cplx<T> w = twl[q * k * TWS];
        if (sign > 0) w.y = -w.y;
        u[q] = cmul(u[q], w);
      }
      bfly<T, RL>(u, sg);
      const int j0 = (i - k) * RL + k;
#pragma unroll
      for (int q = 0; q < RL; ++q) {
        if (!((keep >> (j * RL + q)) & 1ull)) continue;
        const int t = j0 + q * PL;
        const int io = t < pout ? t : t - (N - a.nout);
        T f = a.scale;
        if (a.fac_out) f *= a.fac_out[io];
        out[(o0 * a.nout + io) * a.inner + q0 + b] = u[q] * f;
      }
    }
  }
}

// N > 0: a pass of length N with NB lines per workgroup known at compile time (N * NB / kEPT
// threads); N = 0: any length, from the arguments.
template <typename T, bool CONTIG, int N = 0, int NB = 0>
__device__ __forceinline__ void c2c_body(const cplx<T>* __restrict__ in, cplx<T>* __restrict__ out,
                                         const FftArgs<T>& a, Blk wb) {
  if constexpr (!CONTIG && N > 0) {
    c2c_strided_ct<T, N, NB>(in, out, a, wb);
    return;
  }
  extern __shared__ char smem_raw[];
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
  const int n = N > 0 ? N : a.n, nb = N > 0 ? NB : a.nb, nthr = N > 0 ? N * NB / kEPT : (int)blockDim.x;
  cplx<T>* twl = buf + (CONTIG ? lpad_len(n * nb) : n * nb);
  // occupancy flags of this workgroup's rows (x passes) or of the entries it loads and stores
  // (strided passes), fetched once; the workgroup leaves when nothing it owns is reached by a point
  uint8_t* fld = flag_area(twl, n);
  int64_t o0 = 0, q0 = 0;
  int ncol;
  int need = 0;
  if (CONTIG) {
    // XCD-contiguous numbering only for unmasked passes: with occupancy masks the reached rows cluster,
    // and contiguous ranges would leave some XCDs most of the work
    o0 = (a.rows.m ? wb.x : xcd_linear(wb.x, wb.nx)) * nb;
    ncol = (int)(a.outer - o0 < nb ? a.outer - o0 : nb);
    for (int b = threadIdx.x; b < nb; b += nthr) {
      const uint8_t f = b < ncol && row_needed(a.rows, o0 + b);
      fld[b] = f;
      need |= f;
    }
  } else {
    // plain numbering only where whole lines may be skipped (a line mask): per-entry masks leave
    // every workgroup some work, so neighbours stay on one XCD
    const int64_t lin0 = wb.x + wb.y * wb.nx;
    const int64_t lin = a.line.m ? lin0 : xcd_linear(lin0, wb.nx * wb.ny);
    q0 = (lin % wb.nx) * nb;
    o0 = lin / wb.nx;
    ncol = (int)(a.inner - q0 < nb ? a.inner - q0 : nb);
    const bool line = !a.line.m || a.line.m[mask_index(a.line, o0, 0)];
    for (int i = threadIdx.x; i < a.nin; i += nthr) fld[i] = line && (!a.ld.m || a.ld.m[mask_index(a.ld, o0, i)]);
    need = line;
  }
  if (!__syncthreads_or(need)) return;
  // zero the padding gap [pin, n - (nin - pin))
  const int g0 = a.pin, gl = n - a.nin;
  for (int it = threadIdx.x; it < gl * nb; it += nthr) {
    int t, b;
    if (CONTIG) {
      b = it / gl;
      t = g0 + it - b * gl;
    } else {
      t = g0 + it / nb;
      b = it % nb;
    }
    buf[lidx<CONTIG>(t, b, n, nb)] = mk((T)0, (T)0);
  }
  // load: all global reads of this thread first, then the LDS writes
  cplx<T> v[kEPT];
  int li[kEPT];
  const int nload = a.nin * nb;
#pragma unroll
  for (int j = 0; j < kEPT; ++j) {
    const int e = threadIdx.x + j * nthr;
    li[j] = -1;
    v[j] = mk((T)0, (T)0);
    if (e < nload) {
      int i, b;
      if (CONTIG) {
        b = e / a.nin;
        i = e - b * a.nin;
      } else {
        i = e / nb;
        b = e - i * nb;
      }
      const int t = i < a.pin ? i : n - (a.nin - i);
      li[j] = lidx<CONTIG>(t, b, n, nb);
      const bool use = b < ncol && (CONTIG ? fld[b] : fld[i]);
      if (use) {
        const int64_t gi = CONTIG ? (o0 + b) * a.nin + i : (o0 * a.nin + i) * a.inner + q0 + b;
        v[j] = in[gi];
        if (a.fac_in) v[j] = v[j] * a.fac_in[i];
      }
    }
  }
  // the twiddles' loads go out behind the data loads, so both latencies overlap
  stage_twiddles(a.tw, twl, n);
#pragma unroll
  for (int j = 0; j < kEPT; ++j)
    if (li[j] >= 0) buf[li[j]] = v[j];
  // store flags of this thread's output entries (strided passes), fetched before the stages
  const int nstore = a.nout * nb;
  bool sf[kEPT];
#pragma unroll
  for (int j = 0; j < kEPT; ++j) {
    const int e = threadIdx.x + j * nthr;
    sf[j] = true;
    if (!CONTIG && a.st.m && e < nstore) sf[j] = a.st.m[mask_index(a.st, o0, e / nb)] != 0;
  }
  __syncthreads();
  if constexpr (N > 0)
    stockham_ct<T, CONTIG, N, NB>(buf, twl, a.sign);
  else
    stockham<T, CONTIG>(a, buf, twl, a.nb, a.sign);
#pragma unroll
  for (int j = 0; j < kEPT; ++j) {
    const int e = threadIdx.x + j * nthr;
    if (e >= nstore) continue;
    int i, b;
    if (CONTIG) {
      b = e / a.nout;
      i = e - b * a.nout;
    } else {
      i = e / nb;
      b = e - i * nb;
    }
    if (b >= ncol) continue;
    if (CONTIG ? !fld[b] : !sf[j]) continue;
    const int t = i < a.pout ? i : n - (a.nout - i);
    T f = a.scale;
    if (a.fac_out) f *= a.fac_out[i];
    const int64_t go = CONTIG ? (o0 + b) * a.nout + i : (o0 * a.nout + i) * a.inner + q0 + b;
    out[go] = buf[lidx<CONTIG>(t, b, n, nb)] * f;
  }
}

template <typename T, bool CONTIG, int N = 0, int NB = 0>
__global__ __launch_bounds__(kMaxFftThreads) void k_fft_c2c(const cplx<T>* __restrict__ in,
                                                            cplx<T>* __restrict__ out, FftArgs<T> a) {
  c2c_body<T, CONTIG, N, NB>(in, out, a, launch_blk());
}

// One pass of a launch over parts: its operands and description.
template <typename T>
struct FftIO {
  const void* in;
  void* out;
  FftArgs<T> a;
};

// The lengths and line counts with compile-time passes (the standard line count for each length).
#define FSIB_FFT_CT_LIST(X) X(64, 32) X(96, 16) X(128, 16) X(160, 12) X(192, 8) X(256, 8) X(320, 6) X(384, 4) \
  X(512, 4) X(1024, 2)

// Launches over parts: CT = true when every part has a compile-time (length, line count) pair (the
// kernel then holds only those bodies), else the runtime-length body alone (it needs about twice the
// registers, which would lower the occupancy of the compile-time bodies sharing its kernel).
template <typename T, bool CONTIG, bool CT>
__global__ __launch_bounds__(kMaxFftThreads) void k_fft_c2c_parts(Parts<FftIO<T>> f) {
  Blk b;
  const int g = part_blk(f, b);
  if (g < 0) return;
  const FftIO<T>& io = f.a[g];
  const cplx<T>* in = (const cplx<T>*)io.in;
  cplx<T>* out = (cplx<T>*)io.out;
  if constexpr (CT) {
#define FSIB_C2C_PART(N_, NB_)                        \
  if (io.a.n == N_ && io.a.nb == NB_) {               \
    c2c_body<T, CONTIG, N_, NB_>(in, out, io.a, b);   \
    return;                                           \
  }
    FSIB_FFT_CT_LIST(FSIB_C2C_PART)
#undef FSIB_C2C_PART
  } else {
    c2c_body<T, CONTIG>(in, out, io.a, b);
  }
}

// Real lines along x -> half spectra: lines 2b and 2b+1 form z = a + i b; A_m = (Z_m + conj Z_{n-m})/2,
// B_m = (Z_m - conj Z_{n-m})/(2i) for m < nout.  a.outer = number of real lines, a.nb = pairs per block.
template <typename T, int N = 0, int NB = 0>
__device__ __forceinline__ void r2c_body(const T* __restrict__ in, cplx<T>* __restrict__ out, const FftArgs<T>& a,
                                         Blk wb) {
  extern __shared__ char smem_raw[];
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
  const int n = N > 0 ? N : a.n, nb = N > 0 ? NB : a.nb, nthr = N > 0 ? N * NB / kEPT : (int)blockDim.x;
  cplx<T>* twl = buf + lpad_len(n * nb);
  const int64_t pair0 = (a.rows.m ? wb.x : xcd_linear(wb.x, wb.nx)) * nb;
  uint8_t* fl = flag_area(twl, n);  // rows of this workgroup reached by a point
  int need = 0;
  for (int b = threadIdx.x; b < 2 * nb; b += nthr) {
    const int64_t r = 2 * pair0 + b;
    const uint8_t f = r < a.outer && row_needed(a.rows, r);
    fl[b] = f;
    need |= f;
  }
  if (!__syncthreads_or(need)) return;
  cplx<T> v[kEPT];
#pragma unroll
  for (int j = 0; j < kEPT; ++j) {
    const int e = threadIdx.x + j * nthr;
    v[j] = mk((T)0, (T)0);
    if (e < n * nb) {
      const int b = e / n, t = e - b * n;
      const int64_t r0 = 2 * (pair0 + b), r1 = r0 + 1;
      if (fl[2 * b]) v[j].x = in[r0 * n + t];
      if (fl[2 * b + 1]) v[j].y = in[r1 * n + t];
    }
  }
  stage_twiddles(a.tw, twl, n);  // behind the data loads
#pragma unroll
  for (int j = 0; j < kEPT; ++j) {
    const int e = threadIdx.x + j * nthr;
    if (e < n * nb) buf[lpad(e)] = v[j];  // [b][t] layout: e = b*n + t
  }
  __syncthreads();
  if constexpr (N > 0)
    stockham_ct<T, true, N, NB>(buf, twl, a.sign);
  else
    stockham<T, true>(a, buf, twl, a.nb, a.sign);
#pragma unroll
  for (int j = 0; j < kEPT; ++j) {
    const int e = threadIdx.x + j * nthr;
    if (e >= a.nout * nb) continue;
    const int b = e / a.nout, m = e - b * a.nout;
    const int64_t r0 = 2 * (pair0 + b), r1 = r0 + 1;
    if (r0 >= a.outer) continue;
    const cplx<T> Z = buf[lpad(b * n + m)];
    const cplx<T> Zc = conj(buf[lpad(b * n + (m == 0 ? 0 : n - m))]);
    T f = a.scale * (T)0.5;
    if (a.fac_out) f *= a.fac_out[m];
    const cplx<T> s = Z + Zc, d = Z - Zc;
    if (fl[2 * b]) out[r0 * a.nout + m] = s * f;
    if (fl[2 * b + 1]) out[r1 * a.nout + m] = mk(d.y * f, -d.x * f);
  }
}

template <typename T, int N = 0, int NB = 0>
__global__ __launch_bounds__(kMaxFftThreads) void k_fft_r2c_x(const T* __restrict__ in, cplx<T>* __restrict__ out,
                                                              FftArgs<T> a) {
  r2c_body<T, N, NB>(in, out, a, launch_blk());
}

template <typename T, bool CT>
__global__ __launch_bounds__(kMaxFftThreads) void k_fft_r2c_x_parts(Parts<FftIO<T>> f) {
  Blk b;
  const int g = part_blk(f, b);
  if (g < 0) return;
  const FftIO<T>& io = f.a[g];
  const T* in = (const T*)io.in;
  cplx<T>* out = (cplx<T>*)io.out;
  if constexpr (CT) {
#define FSIB_R2C_PART(N_, NB_)              \
  if (io.a.n == N_ && io.a.nb == NB_) {     \
    r2c_body<T, N_, NB_>(in, out, io.a, b); \
    return;                                 \
  }
    FSIB_FFT_CT_LIST(FSIB_R2C_PART)
#undef FSIB_R2C_PART
  } else {
    r2c_body<T>(in, out, io.a, b);
  }
}

// Half spectra along x (nin entries m = 0..nin-1, the rest zero) -> real lines of length n; two
// lines per complex transform: Z_t = A_t + i B_t with A_{n-m} = conj A_m, then Re/Im of the
// inverse transform.  a.outer = number of real lines, a.nb = pairs per block.
template <typename T, int N = 0, int NB = 0>
__device__ __forceinline__ void c2r_body(const cplx<T>* __restrict__ in, T* __restrict__ out, const FftArgs<T>& a,
                                         Blk wb) {
  extern __shared__ char smem_raw[];
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
  const int n = N > 0 ? N : a.n, nb = N > 0 ? NB : a.nb, nthr = N > 0 ? N * NB / kEPT : (int)blockDim.x;
  cplx<T>* twl = buf + lpad_len(n * nb);
  const int64_t pair0 = (a.rows.m ? wb.x : xcd_linear(wb.x, wb.nx)) * nb;
  uint8_t* fl = flag_area(twl, n);  // rows of this workgroup reached by a point
  int need = 0;
  for (int b = threadIdx.x; b < 2 * nb; b += nthr) {
    const int64_t r = 2 * pair0 + b;
    const uint8_t f = r < a.outer && row_needed(a.rows, r);
    fl[b] = f;
    need |= f;
  }
  if (!__syncthreads_or(need)) return;
  cplx<T> A[kEPT], B[kEPT];
#pragma unroll
  for (int j = 0; j < kEPT; ++j) {
    const int e = threadIdx.x + j * nthr;
    A[j] = mk((T)0, (T)0);
    B[j] = mk((T)0, (T)0);
    if (e < n * nb) {
      const int b = e / n, t = e - b * n;
      const int64_t r0 = 2 * (pair0 + b), r1 = r0 + 1;
      const int m = 2 * t <= n ? t : n - t;
      if (m < a.nin) {
        if (fl[2 * b]) A[j] = in[r0 * a.nin + m];
        if (fl[2 * b + 1]) B[j] = in[r1 * a.nin + m];
      }
    }
  }
  stage_twiddles(a.tw, twl, n);  // behind the data loads
#pragma unroll
  for (int j = 0; j < kEPT; ++j) {
    const int e = threadIdx.x + j * nthr;
    if (e < n * nb) {
      const int t = e % n;
      const bool front = 2 * t <= n;
      const int m = front ? t : n - t;
      cplx<T> x = A[j], y = B[j];
      if (m < a.nin) {
        const T f = a.fac_in ? a.fac_in[m] : (T)1;
        x = x * f;
        y = y * f;
        if (m == 0 || 2 * m == n) {
          x.y = (T)0;
          y.y = (T)0;
        } else if (!front) {
          x = conj(x);
          y = conj(y);
        }
      }
      buf[lpad(e)] = mk(x.x - y.y, x.y + y.x);
    }
  }
  __syncthreads();
  if constexpr (N > 0)
    stockham_ct<T, true, N, NB>(buf, twl, a.sign);
  else
    stockham<T, true>(a, buf, twl, a.nb, a.sign);
#pragma unroll
  for (int j = 0; j < kEPT; ++j) {
    const int e = threadIdx.x + j * nthr;
    if (e >= n * nb) continue;
    const int b = e / n, t = e - b * n;
    const int64_t r0 = 2 * (pair0 + b), r1 = r0 + 1;
    const cplx<T> z = buf[lpad(e)];
    if (fl[2 * b]) out[r0 * n + t] = z.x * a.scale;
    if (fl[2 * b + 1]) out[r1 * n + t] = z.y * a.scale;
  }
}

template <typename T, int N = 0, int NB = 0>
__global__ __launch_bounds__(kMaxFftThreads) void k_fft_c2r_x(const cplx<T>* __restrict__ in, T* __restrict__ out,
                                                              FftArgs<T> a) {
  c2r_body<T, N, NB>(in, out, a, launch_blk());
}

template <typename T, bool CT>
__global__ __launch_bounds__(kMaxFftThreads) void k_fft_c2r_x_parts(Parts<FftIO<T>> f) {
  Blk b;
  const int g = part_blk(f, b);
  if (g < 0) return;
  const FftIO<T>& io = f.a[g];
  const cplx<T>* in = (const cplx<T>*)io.in;
  T* out = (T*)io.out;
  if constexpr (CT) {
#define FSIB_C2R_PART(N_, NB_)              \
  if (io.a.n == N_ && io.a.nb == NB_) {     \
    c2r_body<T, N_, NB_>(in, out, io.a, b); \
    return;                                 \
  }
    FSIB_FFT_CT_LIST(FSIB_C2R_PART)
#undef FSIB_C2R_PART
  } else {
    c2r_body<T>(in, out, io.a, b);
  }
}

template <typename T>
static FftArgs<T> base_args(const Plan& p, int n, int sign, const PassMasks& mk) {
  FftArgs<T> a;
  a.line = mk.line;
  a.ld = mk.ld;
  a.st = mk.st;
  a.rows = mk.rows;
  a.n = n;
  a.nst = radix_plan(n, a.radix);
  a.tw = (const cplx<T>*)p.tw.at(n);
  a.sign = sign;
  a.fac_in = nullptr;
  a.fac_out = nullptr;
  a.scale = (T)1;
  return a;
}

static int gcd_int(int a, int b) {
  while (b) {
    const int t = a % b;
    a = b;
    b = t;
  }
  return a;
}

// Lines per workgroup: n*nb*sizeof(complex) within 32 KiB, n*nb a multiple of kEPT (every thread
// owns kEPT elements), preferring whole wavefronts; `cap` bounds nb (columns that exist).
template <typename T>
static int lines_per_block(int n, int64_t cap) {
  const int budget = kFftWgEntries;
  const int step = kEPT / gcd_int(n, kEPT);  // nb multiple of step -> n*nb multiple of kEPT
  int nb = budget / n;
  if (cap > 0 && nb > cap) nb = (int)cap;
  nb = nb / step * step;
  if (nb < step) nb = step;
  // prefer a whole number of 64-wide wavefronts
  for (int c = nb; c >= step; c -= step)
    if (((int64_t)n * c / kEPT) % 64 == 0) return c;
  return nb;
}

// A (length, line count) pair with compile-time passes.
static bool ct_pass(int n, int nb) {
#define FSIB_CT_PAIR(N_, NB_) if (n == N_ && nb == NB_) return true;
  FSIB_FFT_CT_LIST(FSIB_CT_PAIR)
#undef FSIB_CT_PAIR
  return false;
}
template <typename T>
static bool all_ct(const Parts<FftIO<T>>& f) {
  for (int g = 0; g < f.n; ++g)
    if (!ct_pass(f.a[g].a.n, f.a[g].a.nb)) return false;
  return true;
}

// Arguments, grid, threads and LDS of one strided or contiguous complex pass.
template <typename T>
static PartLaunch<FftIO<T>> c2c_launch(const FftCall& c) {
  const Plan& p = *c.p;
  PartLaunch<FftIO<T>> L;
  FftArgs<T>& a = L.a.a;
  a = base_args<T>(p, c.n, c.sign, c.mk);
  a.inner = c.inner;
  a.outer = c.outer;
  a.nin = c.nin;
  a.pin = c.pin;
  a.nout = c.nout;
  a.pout = c.pout;
  a.fac_in = (const T*)c.fac_in;
  a.fac_out = (const T*)c.fac_out;
  a.scale = (T)c.scale;
  const bool contig = c.inner == 1;
  const int n = c.n;
  a.nb = lines_per_block<T>(n, contig ? c.outer : c.inner);
  L.a.in = c.in;
  L.a.out = c.out;
  L.threads = n * a.nb / kEPT;
  L.lds = (size_t)((contig ? lpad_len(n * a.nb) : n * a.nb) + n) * sizeof(cplx<T>) + flag_bytes(contig ? a.nb : c.nin);
  if (c.outer <= 0 || c.inner <= 0) {
    L.nx = 0;
  } else if (contig) {
    L.nx = (c.outer + a.nb - 1) / a.nb;
  } else {
    L.nx = (c.inner + a.nb - 1) / a.nb;
    L.ny = c.outer;
  }
  return L;
}

template <typename T>
static hipError_t c2c_one(const PartLaunch<FftIO<T>>& L, bool contig, hipStream_t st) {
  const FftArgs<T>& a = L.a.a;
  const int n = a.n;
  const dim3 grid((unsigned)L.nx, (unsigned)L.ny);
  const cplx<T>* in = (const cplx<T>*)L.a.in;
  cplx<T>* out = (cplx<T>*)L.a.out;
  // lengths with compile-time specialisations (when the line count is the standard one for n)
#define FSIB_C2C_CT(N_, NB_)                                                                               \
  if (n == N_ && a.nb == NB_) {                                                                           \
    if (contig)                                                                                           \
      hipLaunchKernelGGL((k_fft_c2c<T, true, N_, NB_>), grid, dim3(L.threads), L.lds, st, in, out, a);    \
    else                                                                                                  \
      hipLaunchKernelGGL((k_fft_c2c<T, false, N_, NB_>), grid, dim3(L.threads), L.lds, st, in, out, a);   \
  } else
  FSIB_FFT_CT_LIST(FSIB_C2C_CT) {
    if (contig)
      hipLaunchKernelGGL((k_fft_c2c<T, true>), grid, dim3(L.threads), L.lds, st, in, out, a);
    else
      hipLaunchKernelGGL((k_fft_c2c<T, false>), grid, dim3(L.threads), L.lds, st, in, out, a);
  }
#undef FSIB_C2C_CT
  return hipGetLastError();
}

template <typename T>
static hipError_t c2c_impl(const FftCall& c, hipStream_t st) {
  const Plan& p = *c.p;
  const PartLaunch<FftIO<T>> L = c2c_launch<T>(c);
  const bool contig = c.inner == 1;
  const bool prof = !contig && prof_on(p, PROF_FFT_STRIDED);
  if (prof) prof_start(p, st);
  const hipError_t e = c2c_one<T>(L, contig, st);
  // algorithmic bytes: every input entry read once, every output entry written once
  if (prof) prof_stop(p, (double)(c.nin + c.nout) * c.inner * c.outer * sizeof(cplx<T>), st);
  return e;
}

// Passes of the plans of a group, one launch for the strided and one for the contiguous ones where
// their workgroup sizes agree.
template <typename T>
static hipError_t c2c_group(const std::vector<FftCall>& calls, hipStream_t st) {
  for (int contig = 0; contig < 2; ++contig) {
    std::vector<PartLaunch<FftIO<T>>> v;
    for (const FftCall& c : calls)
      if ((c.inner == 1) == (contig == 1)) v.push_back(c2c_launch<T>(c));
    const bool ct = contig == 1;
    const hipError_t e = launch_parts(
        v, [&](const PartLaunch<FftIO<T>>& L) { return c2c_one<T>(L, ct, st); },
        [&](const Parts<FftIO<T>>& f, int64_t nwg, size_t lds, int nthr) {
          const dim3 grid((unsigned)nwg), thr(nthr);
          const bool c = all_ct(f);
          if (ct && c) hipLaunchKernelGGL((k_fft_c2c_parts<T, true, true>), grid, thr, lds, st, f);
          else if (ct) hipLaunchKernelGGL((k_fft_c2c_parts<T, true, false>), grid, thr, lds, st, f);
          else if (c) hipLaunchKernelGGL((k_fft_c2c_parts<T, false, true>), grid, thr, lds, st, f);
          else hipLaunchKernelGGL((k_fft_c2c_parts<T, false, false>), grid, thr, lds, st, f);
          return hipGetLastError();
        });
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_fft_c2c_group(const std::vector<FftCall>& calls, hipStream_t st) {
  if (calls.empty()) return hipSuccess;
  return calls[0].p->prec == FSIB_F64 ? c2c_group<double>(calls, st) : c2c_group<float>(calls, st);
}

// One line of length n per workgroup is the smallest launch of every pass: it must fit the thread
// limit (kEPT elements per thread) and the LDS of one workgroup (contiguous layout with padding,
// twiddles and flags; the strided layout with one flag per input entry).
bool fft_line_fits(const Plan& p, int n) {
  if (n > kEPT * kMaxFftThreads) return false;
  const size_t cs = p.prec == FSIB_F64 ? sizeof(cplx<double>) : sizeof(cplx<float>);
  const size_t contig = (size_t)(lpad_len(n) + n) * cs + flag_bytes(2);
  const size_t strided = (size_t)2 * n * cs + flag_bytes(n);
  return std::max(contig, strided) <= (size_t)p.lds_max;
}

hipError_t launch_fft_c2c(const Plan& p, const void* in, void* out, int n, int sign, int64_t inner, int64_t outer,
                          int nin, int pin, int nout, int pout, const void* fac_in, const void* fac_out, double scale,
                          hipStream_t st, const PassMasks& mk) {
  if (outer <= 0 || inner <= 0) return hipSuccess;
  const FftCall c{&p, in, out, n, sign, inner, outer, nin, pin, nout, pout, fac_in, fac_out, scale, mk};
  return p.prec == FSIB_F64 ? c2c_impl<double>(c, st) : c2c_impl<float>(c, st);
}

// Contiguous real-data passes along x: c.outer = real rows; r2c keeps c.nout half-spectrum entries
// (c.fac_out, c.scale), c2r reads c.nin (c.fac_in, c.scale).
template <typename T>
static PartLaunch<FftIO<T>> x_launch(const FftCall& c, bool r2c) {
  const Plan& p = *c.p;
  PartLaunch<FftIO<T>> L;
  FftArgs<T>& a = L.a.a;
  const int n = c.n;
  a = base_args<T>(p, n, r2c ? -1 : +1, c.mk);
  a.inner = 1;
  a.outer = c.outer;
  if (r2c) {
    a.nin = n;
    a.pin = n;
    a.nout = c.nout;
    a.pout = c.nout;
    a.fac_out = (const T*)c.fac_out;
  } else {
    a.nin = c.nin;
    a.pin = c.nin;
    a.nout = n;
    a.pout = n;
    a.fac_in = (const T*)c.fac_in;
  }
  a.scale = (T)c.scale;
  const int64_t pairs = (c.outer + 1) / 2;
  a.nb = lines_per_block<T>(n, pairs);
  L.a.in = c.in;
  L.a.out = c.out;
  L.threads = n * a.nb / kEPT;
  L.lds = (size_t)(lpad_len(n * a.nb) + n) * sizeof(cplx<T>) + flag_bytes(2 * a.nb);
  L.nx = c.outer > 0 ? (pairs + a.nb - 1) / a.nb : 0;
  return L;
}

template <typename T>
static hipError_t x_one(const PartLaunch<FftIO<T>>& L, bool r2c, hipStream_t st) {
  const FftArgs<T>& a = L.a.a;
  const int n = a.n;
  const dim3 grid((unsigned)L.nx);
  if (r2c) {
    const T* in = (const T*)L.a.in;
    cplx<T>* out = (cplx<T>*)L.a.out;
#define FSIB_R2C_CT(N_, NB_) \
  if (n == N_ && a.nb == NB_) hipLaunchKernelGGL((k_fft_r2c_x<T, N_, NB_>), grid, dim3(L.threads), L.lds, st, in, out, a); else
    FSIB_FFT_CT_LIST(FSIB_R2C_CT)
    hipLaunchKernelGGL(k_fft_r2c_x<T>, grid, dim3(L.threads), L.lds, st, in, out, a);
#undef FSIB_R2C_CT
  } else {
    const cplx<T>* in = (const cplx<T>*)L.a.in;
    T* out = (T*)L.a.out;
#define FSIB_C2R_CT(N_, NB_) \
  if (n == N_ && a.nb == NB_) hipLaunchKernelGGL((k_fft_c2r_x<T, N_, NB_>), grid, dim3(L.threads), L.lds, st, in, out, a); else
    FSIB_FFT_CT_LIST(FSIB_C2R_CT)
    hipLaunchKernelGGL(k_fft_c2r_x<T>, grid, dim3(L.threads), L.lds, st, in, out, a);
#undef FSIB_C2R_CT
  }
  return hipGetLastError();
}

template <typename T>
static hipError_t r2c_impl(const Plan& p, const void* in, void* out, int n, int64_t rows, int nout, const void* fout,
                           double scale, hipStream_t st, const PassMasks& mk) {
  const FftCall c{&p, in, out, n, -1, 1, rows, n, n, nout, nout, nullptr, fout, scale, mk};
  const PartLaunch<FftIO<T>> L = x_launch<T>(c, true);
  const bool prof = prof_on(p, PROF_FFT_X);
  if (prof) prof_start(p, st);
  const hipError_t e = x_one<T>(L, true, st);
  if (prof) prof_stop(p, (double)rows * (n * sizeof(T) + nout * sizeof(cplx<T>)), st);
  return e;
}

template <typename T>
static hipError_t c2r_impl(const Plan& p, const void* in, void* out, int n, int64_t rows, int nin, const void* fin,
                           double scale, hipStream_t st, const PassMasks& mk) {
  const FftCall c{&p, in, out, n, +1, 1, rows, nin, nin, n, n, fin, nullptr, scale, mk};
  const PartLaunch<FftIO<T>> L = x_launch<T>(c, false);
  const bool prof = prof_on(p, PROF_FFT_X);
  if (prof) prof_start(p, st);
  const hipError_t e = x_one<T>(L, false, st);
  if (prof) prof_stop(p, (double)rows * (nin * sizeof(cplx<T>) + n * sizeof(T)), st);
  return e;
}

template <typename T>
static hipError_t x_group(const std::vector<FftCall>& calls, bool r2c, hipStream_t st) {
  std::vector<PartLaunch<FftIO<T>>> v;
  for (const FftCall& c : calls) v.push_back(x_launch<T>(c, r2c));
  return launch_parts(
      v, [&](const PartLaunch<FftIO<T>>& L) { return x_one<T>(L, r2c, st); },
      [&](const Parts<FftIO<T>>& f, int64_t nwg, size_t lds, int nthr) {
        const dim3 grid((unsigned)nwg), thr(nthr);
        const bool c = all_ct(f);
        if (r2c && c) hipLaunchKernelGGL((k_fft_r2c_x_parts<T, true>), grid, thr, lds, st, f);
        else if (r2c) hipLaunchKernelGGL((k_fft_r2c_x_parts<T, false>), grid, thr, lds, st, f);
        else if (c) hipLaunchKernelGGL((k_fft_c2r_x_parts<T, true>), grid, thr, lds, st, f);
        else hipLaunchKernelGGL((k_fft_c2r_x_parts<T, false>), grid, thr, lds, st, f);
        return hipGetLastError();
      });
}

hipError_t launch_fft_x_group(const std::vector<FftCall>& calls, bool r2c, hipStream_t st) {
  if (calls.empty()) return hipSuccess;
  return calls[0].p->prec == FSIB_F64 ? x_group<double>(calls, r2c, st) : x_group<float>(calls, r2c, st);
}

hipError_t launch_fft_r2c_x(const Plan& p, const void* in, void* out, int n, int64_t rows, int nout,
                            const void* fac_out, double scale, hipStream_t st, const PassMasks& mk) {
  if (rows <= 0) return hipSuccess;
  return p.prec == FSIB_F64 ? r2c_impl<double>(p, in, out, n, rows, nout, fac_out, scale, st, mk)
                            : r2c_impl<float>(p, in, out, n, rows, nout, fac_out, scale, st, mk);
}

hipError_t launch_fft_c2r_x(const Plan& p, const void* in, void* out, int n, int64_t rows, int nin,
                            const void* fac_in, double scale, hipStream_t st, const PassMasks& mk) {
  if (rows <= 0) return hipSuccess;
  return p.prec == FSIB_F64 ? c2r_impl<double>(p, in, out, n, rows, nin, fac_in, scale, st, mk)
                            : c2r_impl<float>(p, in, out, n, rows, nin, fac_in, scale, st, mk);
}

}  // namespace fsib
