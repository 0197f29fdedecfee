// Last pass of the dealiased products fused with the Navier-Stokes update.
//
// The products pipeline ends with the forward transform along z of the six product spectra
// (u_a u_b)^ (192 dealiasing points down to 128 modes, Sec. 3.1), and the update (Alg. 1 with V-hat
// of Alg. 2) then needs, per mode, shat_a = sum_b i k_b (u_a u_b)^.  Here a workgroup transforms
// the six products of NB neighbouring (ky, kx) columns in turn, keeps the last Stockham stage's
// outputs in registers and adds each product's share of shat to the modes the thread owns; after the
// sixth product it reads fhat and u of those modes and writes the updated u.  The product spectra
// never reach memory: per half step at 128^3 in FP64 that saves writing and reading back six half
// spectra (2 x 102 MB), and a launch.
#include "fft_device.hpp"
#include "fluid_device.hpp"

namespace fsib {

template <typename T>
struct ZFluidArgs {
  const cplx<T>* prod;  // products after the forward y pass: [6][192][N1 * Hx], order xx xy xz yy yz zz
  const cplx<T>* tw;    // tw[t] = exp(-2 pi i t / 192)
  ModeGeo g;
  int mode;  // FLUID_NS_HALF or FLUID_NS_FULL
  T rho, mu, dt;
  T body[3];
  const cplx<T>* fhat;
  const cplx<T>* uin;
  cplx<T>* uout;
};

constexpr int kZfN = 192;    // dealiasing points along z
constexpr int kZfModes = 128;  // modes along z

// s_ca += i k_cb pi and, for ca != cb, s_cb += i k_ca pi
template <typename T>
__device__ __forceinline__ void add_shat(cplx<T>* s, cplx<T> pi, T k0, T k1, T k2, int ca, int cb) {
  const cplx<T> ip = mk(-pi.y, pi.x);
  const T ka = ca == 0 ? k0 : (ca == 1 ? k1 : k2);
  const T kb = cb == 0 ? k0 : (cb == 1 ? k1 : k2);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const T coef = (c == ca ? kb : (T)0) + (c == cb && ca != cb ? ka : (T)0);
    s[c] = s[c] + ip * coef;
  }
}

// The update of one owned mode (index idx of each component) from its shat.
template <typename T>
__device__ __forceinline__ void update_mode(const ZFluidArgs<T>& A, int64_t nm, bool nyq, int64_t idx, T k0, T k1,
                                            T k2v, const cplx<T>* s) {
  if (nyq) {
#pragma unroll
    for (int a = 0; a < 3; ++a) A.uout[a * nm + idx] = mk((T)0, (T)0);
    return;
  }
  const T k[3] = {k0, k1, k2v};
  const T ksq = k0 * k0 + k1 * k1 + k2v * k2v;
  cplx<T> fv[3], uv[3], r[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    fv[a] = A.fhat[a * nm + idx];
    uv[a] = A.uin[a * nm + idx];
  }
  ns_mode_update<T, 3>(A.mode, A.rho, A.mu, A.dt, A.body, k, ksq, s, fv, uv, r);
#pragma unroll
  for (int a = 0; a < 3; ++a) A.uout[a * nm + idx] = r[a];
}

// Thread layout as in the strided passes: first stage (radix 8) butterfly i = tid / NB of column
// b = tid % NB; last stage (radix 3 over thirds of 64) butterflies bf = tid + j NTHR, i = bf / NB,
// whose outputs t = i and t = i + 128 are the modes kz = i and kz = i - 64 (t = i + 64 is dropped by
// the truncation to 128 modes).  With NTHR = 32 NB each thread owns two last-stage butterflies (four
// modes, 12 complex shat accumulators); the first and middle stages leave a quarter of the threads
// idle.  FP64 takes four columns per workgroup (rows of 64 bytes; the neighbouring workgroup, on the
// same XCD, reads the other half of each 128-byte line): 128^3 step 1.107 ms, against 1.111 with 8
// columns, 1.162 with 2, and 1.113 with 4 columns on 64 NB threads (1.157 unfused).  FP32 takes
// eight (rows of 64 bytes again): 0.812 ms against 0.835 with four.
template <typename T, int NB, int NTHR>
__global__ __launch_bounds__(NTHR) void k_products_z_fluid(ZFluidArgs<T> A) {
  constexpr int N = kZfN;
  constexpr int NS = ct_nstages(N);
  constexpr int R0 = ct_radix_at(N, 0), M0 = N / R0;
  constexpr int RL = ct_radix_at(N, NS - 1), PL = ct_p_before(N, NS - 1), ML = N / RL;
  static_assert(M0 * NB <= NTHR, "one first-stage butterfly per thread at most");
  static_assert(RL == 3 && PL == 64 && ML == 64 && kZfModes == 2 * PL, "last stage: radix 3 over thirds of 64");
  constexpr int NBFL = (ML * NB + NTHR - 1) / NTHR;
  extern __shared__ char smem_raw[];
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* twl = buf + N * NB;
  const ModeGeo& g = A.g;
  const int64_t inner = g.N[1] * g.Hx;  // (ky, kx) columns of one z line
  const int64_t nm = inner * kZfModes;   // modes per component
  const int64_t q0 = xcd_linear(blockIdx.x, gridDim.x) * NB;
  const int ncol = (int)(inner - q0 < NB ? inner - q0 : NB);
  const int tid = threadIdx.x;
  const T twopi_L = (T)(6.283185307179586476925286766559 / g.L);
  // columns of the modes this thread owns (their kx, ky are formed where needed)
  int cx[NBFL], cy[NBFL];
#pragma unroll
  for (int j = 0; j < NBFL; ++j) {
    const int bf = tid + j * NTHR, b = bf - (bf / NB) * NB;
    const int64_t c = q0 + (b < ncol ? b : 0);
    cx[j] = (int)(c % g.Hx);
    cy[j] = (int)mode_of(c / g.Hx, g.N[1]);
  }
  cplx<T> sf[NBFL][3], sb[NBFL][3];
#pragma unroll
  for (int j = 0; j < NBFL; ++j)
#pragma unroll
    for (int c = 0; c < 3; ++c) sf[j][c] = sb[j][c] = mk((T)0, (T)0);
  stage_twiddles(A.tw, twl, N);  // ready after the first product's first-stage barrier
#pragma unroll 1
  for (int f = 0; f < 6; ++f) {
    const cplx<T>* in = A.prod + (int64_t)f * N * inner + q0;
    if (M0 * NB == NTHR || tid < M0 * NB) {
      const int i = tid / NB, b = tid - (tid / NB) * NB;
      cplx<T> u[R0];
#pragma unroll
      for (int q = 0; q < R0; ++q) u[q] = b < ncol ? in[(int64_t)(i + q * M0) * inner + b] : mk((T)0, (T)0);
      bfly<T, R0>(u, (T)-1);
#pragma unroll
      for (int q = 0; q < R0; ++q) buf[(i * R0 + q) * NB + b] = u[q];
    }
    __syncthreads();
    middle_stages<T, N, NB, NTHR, 1, NS - 1>(buf, twl, -1);
    const int ca = f < 3 ? 0 : (f < 5 ? 1 : 2);
    const int cb = f < 3 ? f : (f < 5 ? f - 2 : 2);
#pragma unroll
    for (int j = 0; j < NBFL; ++j) {
      const int bf = tid + j * NTHR;
      if (!((ML * NB) % NTHR == 0 || bf < ML * NB)) continue;
      const int i = bf / NB, b = bf - (bf / NB) * NB;
      cplx<T> u[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) u[q] = buf[(i + q * ML) * NB + b];
      u[1] = cmul(u[1], twl[i]);
      u[2] = cmul(u[2], twl[2 * i]);
      bfly<T, 3>(u, (T)-1);
      const T kx = twopi_L * (T)cx[j], ky = twopi_L * (T)cy[j];
      add_shat(sf[j], u[0], kx, ky, twopi_L * (T)i, ca, cb);
      add_shat(sb[j], u[2], kx, ky, twopi_L * (T)(i - PL), ca, cb);
    }
    __syncthreads();  // the next product's first stage overwrites buf
  }
  // the update of the owned modes
#pragma unroll
  for (int j = 0; j < NBFL; ++j) {
    const int bf = tid + j * NTHR;
    if (!((ML * NB) % NTHR == 0 || bf < ML * NB)) continue;
    const int i = bf / NB, b = bf - (bf / NB) * NB;
    if (b >= ncol) continue;
    const int64_t c = q0 + b;
    const int64_t ix = c % g.Hx, iy = c / g.Hx;
    const bool nyq_xy = (g.N[0] % 2 == 0 && ix == g.N[0] / 2) || (g.N[1] % 2 == 0 && mode_of(iy, g.N[1]) == -g.N[1] / 2);
    // front mode kz = i, back mode kz = i - 64 (row i + 64; row 64 is the z Nyquist mode, set to zero)
    const T kx = twopi_L * (T)cx[j], ky = twopi_L * (T)cy[j];
    update_mode<T>(A, nm, nyq_xy, (int64_t)i * inner + c, kx, ky, twopi_L * (T)i, sf[j]);
    update_mode<T>(A, nm, nyq_xy || i == 0, (int64_t)(i + PL) * inner + c, kx, ky, twopi_L * (T)(i - PL), sb[j]);
  }
}

bool products_z_fluid_fits(const Plan& p) {
  return p.dim == 3 && p.ns && p.ninst == 1 && p.nd[2] == kZfN && p.N[2] == kZfModes;
}

template <typename T>
static hipError_t zf_impl(const Plan& p, int mode, const fsib_fluid_params& prm, const void* fhat, const void* uin,
                          void* uout, hipStream_t st) {
  constexpr int NB = sizeof(T) == 8 ? 4 : 8, NTHR = 32 * NB;
  ZFluidArgs<T> A;
  A.prod = (const cplx<T>*)p.D1;
  A.tw = (const cplx<T>*)p.tw.at(kZfN);
  A.g.dim = 3;
  for (int a = 0; a < 3; ++a) A.g.N[a] = p.N[a];
  A.g.Hx = p.Hx;
  A.g.L = p.L;
  A.mode = mode;
  A.rho = (T)prm.rho;
  A.mu = (T)prm.mu;
  A.dt = (T)prm.dt;
  for (int a = 0; a < 3; ++a) A.body[a] = (T)prm.body[a];
  A.fhat = (const cplx<T>*)fhat;
  A.uin = (const cplx<T>*)uin;
  A.uout = (cplx<T>*)uout;
  const int64_t inner = p.N[1] * p.Hx;
  const unsigned nblk = (unsigned)((inner + NB - 1) / NB);
  const size_t lds = (size_t)(kZfN * NB + kZfN) * sizeof(cplx<T>);
  hipLaunchKernelGGL((k_products_z_fluid<T, NB, NTHR>), dim3(nblk), dim3(NTHR), lds, st, A);
  return hipGetLastError();
}

hipError_t launch_products_z_fluid(const Plan& p, int mode, const fsib_fluid_params& prm, const void* fhat,
                                   const void* uin, void* uout, hipStream_t st) {
  return p.prec == FSIB_F64 ? zf_impl<double>(p, mode, prm, fhat, uin, uout, st)
                            : zf_impl<float>(p, mode, prm, fhat, uin, uout, st);
}

}  // namespace fsib
