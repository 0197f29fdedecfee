// Fourier-space fluid update, dealiased products, force laws and FP64 diagnostics.
//
// Fluid update on half spectra (one thread per mode, all components at once):
//   Stokes (Sec. 6.1, eq. stokeslet):  uhat = (fhat - k (k.fhat)/|k|^2) / (mu |k|^2), uhat(0) = 0.
//   Navier-Stokes (Alg. 1 with V-hat of Alg. 2):
//     P = fhat/rho - shat,  Q = P - k (k.P)/|k|^2  (|k|^2 := 1 at k = 0, projection only),
//     half step  u_mid = (dt/2 Q + u)/(1 + a),  full step  u_new = (dt Q + (1 - a) u)/(1 + a),
//     a = mu dt |k|^2 / (2 rho) with the true |k|^2.
//   shat enters in divergence form, shat_a = sum_b i k_b (u_a u_b)^, which equals the advective
//   form of eq. nonlinear_physical for the divergence-free fields the update produces; the
//   products are formed on the dealiasing grid (three-halves rule, Sec. 3.1).
//   Modes with any m_a = -N_a/2 (even N_a) are set to zero so the field stays real.
#include "fluid_device.hpp"
#include "plan.hpp"

namespace fsib {

template <typename T>
struct FluidArgs {
  ModeGeo g;
  int mode;
  T rho, mu, dt, b0, b1, b2;
  const cplx<T>* fhat;
  const cplx<T>* pihat;
  const cplx<T>* uin;
  cplx<T>* uout;
};

template <typename T, int DIM>
__device__ __forceinline__ void fluid_body(const FluidArgs<T>& A, Blk wb) {
  const ModeGeo& g = A.g;
  const int mode = A.mode;
  const T rho = A.rho, mu = A.mu, dt = A.dt, b0 = A.b0, b1 = A.b1, b2 = A.b2;
  const cplx<T>* __restrict__ fhat = A.fhat;
  const cplx<T>* __restrict__ pihat = A.pihat;
  const cplx<T>* uin = A.uin;
  cplx<T>* uout = A.uout;
  const int64_t nm = g.Hx * g.N[1] * (DIM == 3 ? g.N[2] : 1);
  const int64_t idx = wb.x * blockDim.x + threadIdx.x;
  if (idx >= nm) return;
  // instance wb.y of a multi-instance (Stokes) plan: its dim half spectra follow the previous ones
  const int64_t ib = wb.y * DIM * nm;
  fhat += ib;
  uout += ib;
  if (uin) uin += ib;
  const int64_t ix = idx % g.Hx;
  const int64_t iy = (idx / g.Hx) % g.N[1];
  const int64_t iz = DIM == 3 ? idx / (g.Hx * g.N[1]) : 0;
  const int64_t m[3] = {ix, mode_of(iy, g.N[1]), DIM == 3 ? mode_of(iz, g.N[2]) : 0};
  bool nyq = false;
  for (int a = 0; a < DIM; ++a)
    if (g.N[a] % 2 == 0 && (a == 0 ? ix == g.N[0] / 2 : m[a] == -g.N[a] / 2)) nyq = true;
  if (nyq) {
    for (int a = 0; a < DIM; ++a) uout[a * nm + idx] = mk((T)0, (T)0);
    return;
  }
  const T twopi_L = (T)(6.283185307179586476925286766559 / g.L);
  T k[3];
  T k2 = 0;
  for (int a = 0; a < DIM; ++a) {
    k[a] = twopi_L * (T)m[a];
    k2 += k[a] * k[a];
  }
  if (mode == FLUID_STOKES) {
    if (k2 == (T)0) {
      for (int a = 0; a < DIM; ++a) uout[a * nm + idx] = mk((T)0, (T)0);
      return;
    }
    cplx<T> f[3];
    cplx<T> kf = mk((T)0, (T)0);
    for (int a = 0; a < DIM; ++a) {
      f[a] = fhat[a * nm + idx];
      kf = kf + f[a] * k[a];
    }
    const T inv = (T)1 / (mu * k2);
    for (int a = 0; a < DIM; ++a) uout[a * nm + idx] = (f[a] - kf * (k[a] / k2)) * inv;
    return;
  }
  // Navier-Stokes
  cplx<T> sh[3], f[3], u[3], r[3];
  for (int a = 0; a < DIM; ++a) {
    cplx<T> acc = mk((T)0, (T)0);
    for (int b = 0; b < DIM; ++b) acc = acc + mul_i(pihat[sym_index(a, b, DIM) * nm + idx], k[b]);
    sh[a] = acc;
    f[a] = fhat[a * nm + idx];
    u[a] = uin[a * nm + idx];
  }
  const T body[3] = {b0, b1, b2};
  ns_mode_update<T, DIM>(mode, rho, mu, dt, body, k, k2, sh, f, u, r);
  for (int a = 0; a < DIM; ++a) uout[a * nm + idx] = r[a];
}

template <typename T, int DIM>
__global__ void k_fluid(FluidArgs<T> a) { fluid_body<T, DIM>(a, launch_blk()); }
template <typename T, int DIM>
__global__ void k_fluid_parts(Parts<FluidArgs<T>> f) {
  Blk b;
  const int g = part_blk(f, b);
  if (g >= 0) fluid_body<T, DIM>(f.a[g], b);
}

static ModeGeo mode_geo(const Plan& p) {
  ModeGeo g;
  g.dim = p.dim;
  for (int a = 0; a < 3; ++a) g.N[a] = p.N[a];
  g.Hx = p.Hx;
  g.L = p.L;
  return g;
}

template <typename T>
static PartLaunch<FluidArgs<T>> fluid_launch(const Plan& p, int mode, const fsib_fluid_params& prm, const void* fhat,
                                             const void* uin, void* uout) {
  PartLaunch<FluidArgs<T>> L;
  L.a = FluidArgs<T>{mode_geo(p), mode, (T)prm.rho, (T)prm.mu, (T)prm.dt, (T)prm.body[0], (T)prm.body[1],
                     (T)prm.body[2], (const cplx<T>*)fhat, (const cplx<T>*)p.pihat, (const cplx<T>*)uin,
                     (cplx<T>*)uout};
  L.nx = (p.modes_half() + 255) / 256;
  L.ny = p.ninst;  // one row of blocks per instance
  return L;
}

template <typename T, int DIM>
static hipError_t fluid_one(const PartLaunch<FluidArgs<T>>& L, hipStream_t st) {
  hipLaunchKernelGGL((k_fluid<T, DIM>), dim3((unsigned)L.nx, (unsigned)L.ny), dim3(256), 0, st, L.a);
  return hipGetLastError();
}

hipError_t launch_fluid_update(const Plan& p, int mode, const fsib_fluid_params& prm, const void* fhat,
                               const void* uin, void* uout, hipStream_t st) {
  if (p.prec == FSIB_F64) {
    const auto L = fluid_launch<double>(p, mode, prm, fhat, uin, uout);
    return p.dim == 3 ? fluid_one<double, 3>(L, st) : fluid_one<double, 2>(L, st);
  }
  const auto L = fluid_launch<float>(p, mode, prm, fhat, uin, uout);
  return p.dim == 3 ? fluid_one<float, 3>(L, st) : fluid_one<float, 2>(L, st);
}

template <typename T, int DIM>
static hipError_t fluid_stokes_group(const std::vector<Plan*>& ps, const fsib_fluid_params* prm, void* const* uhat,
                                     hipStream_t st) {
  std::vector<PartLaunch<FluidArgs<T>>> v(ps.size());
  for (size_t g = 0; g < ps.size(); ++g) v[g] = fluid_launch<T>(*ps[g], FLUID_STOKES, prm[g], ps[g]->fhat, nullptr, uhat[g]);
  return launch_parts(
      v, [&](const PartLaunch<FluidArgs<T>>& L) { return fluid_one<T, DIM>(L, st); },
      [&](const Parts<FluidArgs<T>>& f, int64_t nwg, size_t, int) {
        hipLaunchKernelGGL((k_fluid_parts<T, DIM>), dim3((unsigned)nwg), dim3(256), 0, st, f);
        return hipGetLastError();
      });
}

// The Stokes update of every plan of a group (uhat[g] from plan g's fhat with prm[g]), one launch.
hipError_t launch_fluid_stokes_group(const std::vector<Plan*>& ps, const fsib_fluid_params* prm, void* const* uhat,
                                     hipStream_t st) {
  const bool f64 = ps[0]->prec == FSIB_F64;
  if (ps[0]->dim == 3)
    return f64 ? fluid_stokes_group<double, 3>(ps, prm, uhat, st) : fluid_stokes_group<float, 3>(ps, prm, uhat, st);
  return f64 ? fluid_stokes_group<double, 2>(ps, prm, uhat, st) : fluid_stokes_group<float, 2>(ps, prm, uhat, st);
}

template <typename T, int DIM>
__global__ void k_pressure(ModeGeo g, int ns, T rho, const cplx<T>* __restrict__ fhat,
                           const cplx<T>* __restrict__ pihat, cplx<T>* __restrict__ phat) {
  const int64_t nm = g.Hx * g.N[1] * (DIM == 3 ? g.N[2] : 1);
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nm) return;
  const int64_t ix = idx % g.Hx;
  const int64_t iy = (idx / g.Hx) % g.N[1];
  const int64_t iz = DIM == 3 ? idx / (g.Hx * g.N[1]) : 0;
  const int64_t m[3] = {ix, mode_of(iy, g.N[1]), DIM == 3 ? mode_of(iz, g.N[2]) : 0};
  bool nyq = false;
  for (int a = 0; a < DIM; ++a)
    if (g.N[a] % 2 == 0 && (a == 0 ? ix == g.N[0] / 2 : m[a] == -g.N[a] / 2)) nyq = true;
  const T twopi_L = (T)(6.283185307179586476925286766559 / g.L);
  T k[3];
  T k2 = 0;
  for (int a = 0; a < DIM; ++a) {
    k[a] = twopi_L * (T)m[a];
    k2 += k[a] * k[a];
  }
  if (nyq || k2 == (T)0) {
    phat[idx] = mk((T)0, (T)0);
    return;
  }
  cplx<T> kg = mk((T)0, (T)0);
  for (int a = 0; a < DIM; ++a) {
    cplx<T> ga = fhat[a * nm + idx];
    if (ns) {
      cplx<T> s = mk((T)0, (T)0);
      for (int b = 0; b < DIM; ++b) s = s + mul_i(pihat[sym_index(a, b, DIM) * nm + idx], k[b]);
      ga = ga - s * rho;
    }
    kg = kg + ga * k[a];
  }
  phat[idx] = mul_i(kg, -(T)1 / k2);
}

hipError_t launch_pressure(const Plan& p, int ns, double rho, const void* fhat, void* phat, hipStream_t st) {
  ModeGeo g;
  g.dim = p.dim;
  for (int a = 0; a < 3; ++a) g.N[a] = p.N[a];
  g.Hx = p.Hx;
  g.L = p.L;
  const int64_t nm = p.modes_half();
  const unsigned nblk = (unsigned)((nm + 255) / 256);
  if (p.prec == FSIB_F64) {
    using T = double;
    if (p.dim == 3)
      hipLaunchKernelGGL((k_pressure<T, 3>), dim3(nblk), dim3(256), 0, st, g, ns, (T)rho, (const cplx<T>*)fhat,
                         (const cplx<T>*)p.pihat, (cplx<T>*)phat);
    else
      hipLaunchKernelGGL((k_pressure<T, 2>), dim3(nblk), dim3(256), 0, st, g, ns, (T)rho, (const cplx<T>*)fhat,
                         (const cplx<T>*)p.pihat, (cplx<T>*)phat);
  } else {
    using T = float;
    if (p.dim == 3)
      hipLaunchKernelGGL((k_pressure<T, 3>), dim3(nblk), dim3(256), 0, st, g, ns, (T)rho, (const cplx<T>*)fhat,
                         (const cplx<T>*)p.pihat, (cplx<T>*)phat);
    else
      hipLaunchKernelGGL((k_pressure<T, 2>), dim3(nblk), dim3(256), 0, st, g, ns, (T)rho, (const cplx<T>*)fhat,
                         (const cplx<T>*)p.pihat, (cplx<T>*)phat);
  }
  return hipGetLastError();
}

// ---- force laws (double) ----

// Closed curve, Sec. 6.2.1 eq. elstic_force_2d: F_j = K (X_{j+1} + X_{j-1} - 2 X_j) / dtheta^2.
__global__ void k_force_curve(int64_t M, const double* __restrict__ X, double K, double* __restrict__ F) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  const int64_t jp = j + 1 == M ? 0 : j + 1, jm = j == 0 ? M - 1 : j - 1;
  const double dth = 6.283185307179586476925286766559 / (double)M;
  const double c = K / (dth * dth);
  for (int a = 0; a < 2; ++a) F[j * 2 + a] = c * (X[jp * 2 + a] + X[jm * 2 + a] - 2.0 * X[j * 2 + a]);
}

// Surface tension, Sec. 6.2.3: F_i = -(gamma/2) sum over incident triangles (i, j, k) (in the
// triangle's cyclic order starting at i) of (X_j - X_k) x n, n the unit normal of (X_i, X_j, X_k).
// A workgroup takes 32 vertices.  Their incident triangles (entries of the vertex -> triangle CSR)
// are spread evenly over the workgroup's 256 lanes, four per lane with their loads issued together,
// and each triangle's term goes to LDS; then eight lanes per vertex sum its terms, lane l the terms
// l, l + 8, ... in order, and a fixed butterfly sums the lanes.  The per-triangle work is thus
// balanced whatever the degrees: a polar fan vertex of a lat-long mesh (about 200 triangles) no
// longer holds its workgroup for seven rounds of dependent loads (the 40,000-vertex ellipsoid: 27.9
// -> 9 us).  A workgroup whose vertices have more than kSurfTris triangles in all takes them per
// vertex instead (eight lanes per vertex, the same summation order).
// S64 / S32 (nullable): the strengths S = F (quadrature weight 1) in the plan precision, written in
// the same pass.  UK = 1 or 2: the force is taken at X + a U (U in FP64 or FP32), positions the kernel
// forms as it reads them and also writes to Xh, so the half-step move and the force are one pass.
constexpr int kSurfLanes = 8;
constexpr int kSurfThreads = 256;
constexpr int kSurfVerts = kSurfThreads / kSurfLanes;  // vertices per workgroup
constexpr int kSurfTris = 4 * kSurfThreads;           // triangle terms a workgroup holds in LDS
struct SurfaceArgs {
  int64_t M;
  const double* X;
  const void* U;  // UK > 0
  double a;
  double* Xh;     // UK > 0
  double gamma;
  const int32_t* tris;
  const int32_t* ptr;
  const int32_t* idx;
  double* F;
  double* S64;
  float* S32;
};

template <int UK>
__device__ __forceinline__ double surf_pos(const SurfaceArgs& A, int64_t v, int c) {
  const double x = A.X[3 * v + c];
  if constexpr (UK == 1) return fma(A.a, ((const double*)A.U)[3 * v + c], x);  // as k_axpy_pos
  if constexpr (UK == 2) return fma(A.a, (double)((const float*)A.U)[3 * v + c], x);
  return x;
}

// The other two corners (j, k) of triangle t in its cyclic order starting at vertex i.
__device__ __forceinline__ void surf_corners(const SurfaceArgs& A, int t, int i, int& j, int& k) {
  const int v0 = A.tris[3 * t], v1 = A.tris[3 * t + 1], v2 = A.tris[3 * t + 2];
  if (v0 == i) {
    j = v1;
    k = v2;
  } else if (v1 == i) {
    j = v2;
    k = v0;
  } else {
    j = v0;
    k = v1;
  }
}

// The term (X_j - X_k) x n of triangle (i, j, k), X_i = (xi, yi, zi).
template <int UK>
__device__ __forceinline__ void surf_term(const SurfaceArgs& A, int j, int k, double xi, double yi, double zi,
                                          double& t0, double& t1, double& t2) {
  const double ax = surf_pos<UK>(A, j, 0) - xi, ay = surf_pos<UK>(A, j, 1) - yi, az = surf_pos<UK>(A, j, 2) - zi;
  const double bx = surf_pos<UK>(A, k, 0) - xi, by = surf_pos<UK>(A, k, 1) - yi, bz = surf_pos<UK>(A, k, 2) - zi;
  double nx = ay * bz - az * by, ny = az * bx - ax * bz, nz = ax * by - ay * bx;
  const double nn = sqrt(nx * nx + ny * ny + nz * nz);
  if (nn > 0) {
    nx /= nn;
    ny /= nn;
    nz /= nn;
  }
  const double dx = ax - bx, dy = ay - by, dz = az - bz;  // X_j - X_k
  t0 = dy * nz - dz * ny;
  t1 = dz * nx - dx * nz;
  t2 = dx * ny - dy * nx;
}

template <int UK>
__global__ __launch_bounds__(kSurfThreads) void k_force_surface(SurfaceArgs A) {
  __shared__ int s_beg[kSurfVerts + 1];    // the workgroup's terms: vertex s owns [s_beg[s], s_beg[s + 1])
  __shared__ int s_ptr[kSurfVerts];        // CSR offset of each vertex's first triangle
  __shared__ double s_pos[kSurfVerts][3];  // (moved) vertex positions
  __shared__ double s_term[3][kSurfTris];
  const int tid = threadIdx.x;
  const int64_t v0 = (int64_t)blockIdx.x * kSurfVerts;
  // degrees and their prefix sums (wavefront 0: one lane per vertex, a shuffle scan)
  if (tid < 64) {
    const int64_t v = v0 + tid;
    int deg = 0;
    if (tid < kSurfVerts && v < A.M) {
      const int p0 = A.ptr[v];
      deg = A.ptr[v + 1] - p0;
      s_ptr[tid] = p0;
      s_pos[tid][0] = surf_pos<UK>(A, v, 0);
      s_pos[tid][1] = surf_pos<UK>(A, v, 1);
      s_pos[tid][2] = surf_pos<UK>(A, v, 2);
    }
    int incl = deg;
#pragma unroll
    for (int off = 1; off < kSurfVerts; off <<= 1) {
      const int y = __shfl_up(incl, off, 64);
      if ((tid & 63) >= off) incl += y;
    }
    if (tid < kSurfVerts) s_beg[tid + 1] = incl;
    if (tid == 0) s_beg[0] = 0;
  }
  __syncthreads();
  const int total = s_beg[kSurfVerts];
  const int vs = tid / kSurfLanes, lane = tid % kSurfLanes;
  const int64_t i = v0 + vs;
  double f0 = 0, f1 = 0, f2 = 0;
  if (total <= kSurfTris) {
    // every term of the workgroup: entry e of vertex s (upper bound of e in s_beg), four per lane
    int jj[4], kk[4], ss[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = tid + u * kSurfThreads;
      ss[u] = -1;
      if (e < total) {
        int lo = 0, hi = kSurfVerts;  // the last s with s_beg[s] <= e
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (s_beg[mid] <= e) lo = mid;
          else hi = mid;
        }
        ss[u] = lo;
        const int t = A.idx[s_ptr[lo] + (e - s_beg[lo])];
        surf_corners(A, t, (int)(v0 + lo), jj[u], kk[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (ss[u] < 0) continue;
      const int e = tid + u * kSurfThreads;
      double t0, t1, t2;
      surf_term<UK>(A, jj[u], kk[u], s_pos[ss[u]][0], s_pos[ss[u]][1], s_pos[ss[u]][2], t0, t1, t2);
      s_term[0][e] = t0;
      s_term[1][e] = t1;
      s_term[2][e] = t2;
    }
    __syncthreads();
    const int e1 = s_beg[vs + 1];
    for (int e = s_beg[vs] + lane; e < e1; e += kSurfLanes) {
      f0 += s_term[0][e];
      f1 += s_term[1][e];
      f2 += s_term[2][e];
    }
  } else if (i < A.M) {
    // per vertex: lane l takes the vertex's triangles l, l + 8, ..., four per round
    const double xi = s_pos[vs][0], yi = s_pos[vs][1], zi = s_pos[vs][2];
    const int e1 = s_ptr[vs] + (s_beg[vs + 1] - s_beg[vs]);
    for (int e0 = s_ptr[vs] + lane; e0 < e1; e0 += 4 * kSurfLanes) {
      int jj[4], kk[4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (e0 + u * kSurfLanes < e1) surf_corners(A, A.idx[e0 + u * kSurfLanes], (int)i, jj[u], kk[u]);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (e0 + u * kSurfLanes >= e1) continue;
        double t0, t1, t2;
        surf_term<UK>(A, jj[u], kk[u], xi, yi, zi, t0, t1, t2);
        f0 += t0;
        f1 += t1;
        f2 += t2;
      }
    }
  }
#pragma unroll
  for (int off = kSurfLanes / 2; off > 0; off >>= 1) {
    f0 += __shfl_xor(f0, off, 64);
    f1 += __shfl_xor(f1, off, 64);
    f2 += __shfl_xor(f2, off, 64);
  }
  if (lane == 0 && i < A.M) {
    const double g0 = -0.5 * A.gamma * f0, g1 = -0.5 * A.gamma * f1, g2 = -0.5 * A.gamma * f2;
    A.F[3 * i] = g0;
    A.F[3 * i + 1] = g1;
    A.F[3 * i + 2] = g2;
    if (A.S64) {
      A.S64[3 * i] = g0;
      A.S64[3 * i + 1] = g1;
      A.S64[3 * i + 2] = g2;
    }
    if (A.S32) {
      A.S32[3 * i] = (float)g0;
      A.S32[3 * i + 1] = (float)g1;
      A.S32[3 * i + 2] = (float)g2;
    }
    if (UK > 0) {
      A.Xh[3 * i] = s_pos[vs][0];
      A.Xh[3 * i + 1] = s_pos[vs][1];
      A.Xh[3 * i + 2] = s_pos[vs][2];
    }
  }
}

static hipError_t launch_surface(const SurfaceArgs& A, int uk, hipStream_t st) {
  const unsigned nblk = (unsigned)((A.M + kSurfVerts - 1) / kSurfVerts);
  if (uk == 1)
    hipLaunchKernelGGL(k_force_surface<1>, dim3(nblk), dim3(kSurfThreads), 0, st, A);
  else if (uk == 2)
    hipLaunchKernelGGL(k_force_surface<2>, dim3(nblk), dim3(kSurfThreads), 0, st, A);
  else
    hipLaunchKernelGGL(k_force_surface<0>, dim3(nblk), dim3(kSurfThreads), 0, st, A);
  return hipGetLastError();
}

// Edge springs (Sec. 6.2.3, elastic sphere): F_i = K sum_{j linked with i} K_ij (X_j - X_i) over the
// vertex's neighbour list (CSR), K_ij stored per entry.  Linear in X, so it also serves as its own
// Jacobian product.
__global__ void k_force_springs(int64_t M, int dim, const double* __restrict__ X, double K,
                                const int32_t* __restrict__ ptr, const int32_t* __restrict__ nbr,
                                const double* __restrict__ kij, double* __restrict__ F) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  double f[3] = {0, 0, 0};
  for (int e = ptr[i]; e < ptr[i + 1]; ++e) {
    const int64_t j = nbr[e];
    const double k = kij[e];
    for (int a = 0; a < dim; ++a) f[a] += k * (X[j * dim + a] - X[i * dim + a]);
  }
  for (int a = 0; a < dim; ++a) F[i * dim + a] = K * f[a];
}

// Edge stiffness of the elastic sphere from its reference configuration X0 (Sec. 6.2.3), for sigma = 1:
// entry (i -> j) of the neighbour CSR receives, from every triangle (i, j, k) holding edge ij,
// (a0^2 + b0^2 - c0^2) / (8 S0) with c0 = |X_i - X_j|, a0, b0 the other two sides and S0 the area
// (the cotangent of the angle at k, halved).  One thread per vertex, over its incident triangles.
__global__ void k_spring_stiffness(int64_t M, const double* __restrict__ X0, const int32_t* __restrict__ tris,
                                   const int32_t* __restrict__ v2t_ptr, const int32_t* __restrict__ v2t_idx,
                                   const int32_t* __restrict__ nptr, const int32_t* __restrict__ nbr,
                                   double* __restrict__ kij, int* __restrict__ missing) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  const int e0 = nptr[i], e1 = nptr[i + 1];
  for (int e = e0; e < e1; ++e) kij[e] = 0.0;
  for (int q = v2t_ptr[i]; q < v2t_ptr[i + 1]; ++q) {
    const int t = v2t_idx[q];
    const int v[3] = {tris[3 * t], tris[3 * t + 1], tris[3 * t + 2]};
    const int r = v[0] == i ? 0 : (v[1] == i ? 1 : 2);
    const int j = v[(r + 1) % 3], k = v[(r + 2) % 3];
    double dij[3], dik[3], djk[3];
    for (int a = 0; a < 3; ++a) {
      dij[a] = X0[3 * j + a] - X0[3 * i + a];
      dik[a] = X0[3 * k + a] - X0[3 * i + a];
      djk[a] = X0[3 * k + a] - X0[3 * j + a];
    }
    const double cx = dij[1] * dik[2] - dij[2] * dik[1], cy = dij[2] * dik[0] - dij[0] * dik[2],
                 cz = dij[0] * dik[1] - dij[1] * dik[0];
    const double S0 = 0.5 * sqrt(cx * cx + cy * cy + cz * cz);
    const double lij = dij[0] * dij[0] + dij[1] * dij[1] + dij[2] * dij[2];
    const double lik = dik[0] * dik[0] + dik[1] * dik[1] + dik[2] * dik[2];
    const double ljk = djk[0] * djk[0] + djk[1] * djk[1] + djk[2] * djk[2];
    const double kij_t = (ljk + lik - lij) / (8.0 * S0);  // edge ij, opposite k
    const double kik_t = (ljk + lij - lik) / (8.0 * S0);  // edge ik, opposite j
    bool fj = false, fk = false;
    for (int e = e0; e < e1; ++e) {
      if (nbr[e] == j) {
        kij[e] += kij_t;
        fj = true;
      } else if (nbr[e] == k) {
        kij[e] += kik_t;
        fk = true;
      }
    }
    if (!fj || !fk) missing[0] = 1;
  }
}

hipError_t launch_spring_stiffness(int64_t M, const double* X0, const int32_t* tris, const int32_t* v2t_ptr,
                                   const int32_t* v2t_idx, const int32_t* nptr, const int32_t* nbr, double* kij,
                                   int* missing, hipStream_t st) {
  if (M <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_spring_stiffness, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, st, M, X0, tris, v2t_ptr,
                     v2t_idx, nptr, nbr, kij, missing);
  return hipGetLastError();
}

// Target points (Sec. 6.2.2, channel walls): F_i = K (Xtarget_i - X_i); sign = -1 with Xtarget = NULL
// gives the Jacobian product -K V.
__global__ void k_force_target(int64_t n, const double* __restrict__ X, const double* __restrict__ tgt, double K,
                               double* __restrict__ F) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  F[e] = K * ((tgt ? tgt[e] : 0.0) - X[e]);
}

// The closed-curve force for the instances of a multi-instance plan: point j belongs to instance i with
// points [off[i], off[i+1]), whose curve closes on itself and has dtheta = 2 pi / (off[i+1] - off[i]).
__global__ void k_force_curve_inst(int64_t M, const double* __restrict__ X, double K, const int64_t* __restrict__ off,
                                   int ninst, double* __restrict__ F) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  int lo = 0, hi = ninst;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= j) lo = mid;
    else hi = mid;
  }
  const int64_t s = off[lo], e = off[lo + 1];
  const int64_t jp = j + 1 == e ? s : j + 1, jm = j == s ? e - 1 : j - 1;
  const double dth = 6.283185307179586476925286766559 / (double)(e - s);
  const double c = K / (dth * dth);
  for (int a = 0; a < 2; ++a) F[j * 2 + a] = c * (X[jp * 2 + a] + X[jm * 2 + a] - 2.0 * X[j * 2 + a]);
}

// Strengths S = w F per instance: w = 2 pi / M_i (closed curves), with M_i the instance's point count.
template <typename T>
__global__ void k_strengths_inst(int64_t M, int dim, const double* __restrict__ F, const int64_t* __restrict__ off,
                                 int ninst, T* __restrict__ S) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  int lo = 0, hi = ninst;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= j) lo = mid;
    else hi = mid;
  }
  const double w = 6.283185307179586476925286766559 / (double)(off[lo + 1] - off[lo]);
  for (int a = 0; a < dim; ++a) S[j * dim + a] = (T)(w * F[j * dim + a]);
}

// Closed-curve force and its weighted strengths in one pass, for a launch over the plans of a group:
// point j of instance [s, e) (the plan's instance offsets, or the whole range on a one-instance plan)
// gets F_j = K (X_{j+1} + X_{j-1} - 2 X_j) / dtheta^2 with dtheta = 2 pi / (e - s), and S_j = (2 pi / (e - s)) F_j
// in the plan precision -- the values k_force_curve(_inst) and k_strengths(_inst) give.
template <typename T>
struct CurveArgs {
  int64_t M;
  const double* X;
  double K;
  const int64_t* off;  // ninst + 1 offsets, or nullptr: one curve
  int ninst;
  double* F;
  T* S;
};
template <typename T>
__device__ __forceinline__ void curve_force_strengths(const CurveArgs<T>& A, Blk wb) {
  const int64_t j = wb.x * blockDim.x + threadIdx.x;
  if (j >= A.M) return;
  int64_t s = 0, e = A.M;
  if (A.off) {
    int lo = 0, hi = A.ninst;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (A.off[mid] <= j) lo = mid;
      else hi = mid;
    }
    s = A.off[lo];
    e = A.off[lo + 1];
  }
  const int64_t jp = j + 1 == e ? s : j + 1, jm = j == s ? e - 1 : j - 1;
  const double dth = 6.283185307179586476925286766559 / (double)(e - s);
  const double c = A.K / (dth * dth);
  const double w = 6.283185307179586476925286766559 / (double)(e - s);
  for (int a = 0; a < 2; ++a) {
    const double F = c * (A.X[jp * 2 + a] + A.X[jm * 2 + a] - 2.0 * A.X[j * 2 + a]);
    A.F[j * 2 + a] = F;
    A.S[j * 2 + a] = (T)(w * F);
  }
}
template <typename T>
__global__ void k_curve_force_strengths(CurveArgs<T> a) { curve_force_strengths<T>(a, launch_blk()); }
template <typename T>
__global__ void k_curve_force_strengths_parts(Parts<CurveArgs<T>> f) {
  Blk b;
  const int g = part_blk(f, b);
  if (g >= 0) curve_force_strengths<T>(f.a[g], b);
}

hipError_t launch_force(const fsib_force& f, int dim, int64_t M, const double* X, double* F, hipStream_t st) {
  if (M <= 0) return hipSuccess;
  const unsigned nblk = (unsigned)((M + 255) / 256);
  if (f.kind == FSIB_FORCE_CURVE_TENSION)
    hipLaunchKernelGGL(k_force_curve, dim3(nblk), dim3(256), 0, st, M, X, f.K, F);
  else if (f.kind == FSIB_FORCE_EDGE_SPRINGS)
    hipLaunchKernelGGL(k_force_springs, dim3(nblk), dim3(256), 0, st, M, dim, X, f.K, f.v2t_ptr, f.v2t_idx, f.aux, F);
  else if (f.kind == FSIB_FORCE_TARGET)
    hipLaunchKernelGGL(k_force_target, dim3((unsigned)((M * dim + 255) / 256)), dim3(256), 0, st, M * dim, X, f.aux,
                       f.K, F);
  else
    return launch_surface(SurfaceArgs{M, X, nullptr, 0.0, nullptr, f.K, f.tris, f.v2t_ptr, f.v2t_idx, F, nullptr,
                                      nullptr},
                          0, st);
  return hipGetLastError();
}

// Directional derivative dF(X)[V] of the surface-tension force (Sec. 6.2.3), one wavefront per vertex
// (lane l takes the incident triangles l, l + 64, ...).  Per incident triangle (i, j, k): a = X_j - X_i, b = X_k - X_i, m = a x b,
// n = m/|m|; d(a - b) = V_j - V_k, dm = da x b + a x db, dn = (dm - n (n.dm))/|m|, and the force term
// (a - b) x n changes by d(a - b) x n + (a - b) x dn.  F is minus gamma times the gradient of the area,
// so its Jacobian is symmetric and this is also the transpose product the adjoint needs.
__global__ __launch_bounds__(256) void k_force_surface_jvp(int64_t M, const double* __restrict__ X,
                                                           const double* __restrict__ V, double gamma,
                                                           const int32_t* __restrict__ tris,
                                                           const int32_t* __restrict__ ptr,
                                                           const int32_t* __restrict__ idx, double* __restrict__ out) {
  const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (i >= M) return;  // uniform per wavefront
  double f0 = 0, f1 = 0, f2 = 0;
  const double xi = X[3 * i], yi = X[3 * i + 1], zi = X[3 * i + 2];
  const double vxi = V[3 * i], vyi = V[3 * i + 1], vzi = V[3 * i + 2];
  for (int e = ptr[i] + lane; e < ptr[i + 1]; e += 64) {
    const int t = idx[e];
    const int v0 = tris[3 * t], v1 = tris[3 * t + 1], v2 = tris[3 * t + 2];
    int j, k;
    if (v0 == i) {
      j = v1;
      k = v2;
    } else if (v1 == i) {
      j = v2;
      k = v0;
    } else {
      j = v0;
      k = v1;
    }
    const double ax = X[3 * j] - xi, ay = X[3 * j + 1] - yi, az = X[3 * j + 2] - zi;
    const double bx = X[3 * k] - xi, by = X[3 * k + 1] - yi, bz = X[3 * k + 2] - zi;
    const double dax = V[3 * j] - vxi, day = V[3 * j + 1] - vyi, daz = V[3 * j + 2] - vzi;
    const double dbx = V[3 * k] - vxi, dby = V[3 * k + 1] - vyi, dbz = V[3 * k + 2] - vzi;
    const double mx = ay * bz - az * by, my = az * bx - ax * bz, mz = ax * by - ay * bx;
    const double mm = sqrt(mx * mx + my * my + mz * mz);
    if (!(mm > 0)) continue;  // degenerate triangle: its force term is zero, so is the derivative
    const double nx = mx / mm, ny = my / mm, nz = mz / mm;
    // dm = da x b + a x db
    const double dmx = (day * bz - daz * by) + (ay * dbz - az * dby);
    const double dmy = (daz * bx - dax * bz) + (az * dbx - ax * dbz);
    const double dmz = (dax * by - day * bx) + (ax * dby - ay * dbx);
    const double nd = nx * dmx + ny * dmy + nz * dmz;
    const double dnx = (dmx - nx * nd) / mm, dny = (dmy - ny * nd) / mm, dnz = (dmz - nz * nd) / mm;
    const double ex = ax - bx, ey = ay - by, ez = az - bz;          // X_j - X_k
    const double dex = dax - dbx, dey = day - dby, dez = daz - dbz;  // V_j - V_k
    f0 += (dey * nz - dez * ny) + (ey * dnz - ez * dny);
    f1 += (dez * nx - dex * nz) + (ez * dnx - ex * dnz);
    f2 += (dex * ny - dey * nx) + (ex * dny - ey * dnx);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    f0 += __shfl_xor(f0, off, 64);
    f1 += __shfl_xor(f1, off, 64);
    f2 += __shfl_xor(f2, off, 64);
  }
  if (lane == 0) {
    out[3 * i] = -0.5 * gamma * f0;
    out[3 * i + 1] = -0.5 * gamma * f1;
    out[3 * i + 2] = -0.5 * gamma * f2;
  }
}

hipError_t launch_force_jvp(const fsib_force& f, int dim, int64_t M, const double* X, const double* V, double* out,
                            hipStream_t st) {
  if (M <= 0) return hipSuccess;
  if (f.kind == FSIB_FORCE_CURVE_TENSION)  // the curve force is linear in X: dF(X)[V] = F(V)
    hipLaunchKernelGGL(k_force_curve, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, st, M, V, f.K, out);
  else if (f.kind == FSIB_FORCE_EDGE_SPRINGS)  // linear too
    hipLaunchKernelGGL(k_force_springs, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, st, M, dim, V, f.K, f.v2t_ptr,
                       f.v2t_idx, f.aux, out);
  else if (f.kind == FSIB_FORCE_TARGET)  // dF[V] = -K V
    hipLaunchKernelGGL(k_force_target, dim3((unsigned)((M * dim + 255) / 256)), dim3(256), 0, st, M * dim, V,
                       (const double*)nullptr, f.K, out);
  else
    hipLaunchKernelGGL(k_force_surface_jvp, dim3((unsigned)((M + 3) / 4)), dim3(256), 0, st, M, X, V, f.K, f.tris,
                       f.v2t_ptr, f.v2t_idx, out);
  return hipGetLastError();
}

// Strengths S_j = w_j F_j in the plan precision (quadrature weights of eq. force_spreading_quad).
template <typename T>
__global__ void k_strengths(int64_t n, const double* __restrict__ F, double w, T* __restrict__ S) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) S[i] = (T)(w * F[i]);
}

double force_weight(int kind, int64_t M) {
  if (kind != FSIB_FORCE_CURVE_TENSION) return 1.0;
  return M > 0 ? 6.283185307179586476925286766559 / (double)M : 0.0;
}

hipError_t launch_force_plan(const Plan& p, const fsib_force& f, int64_t M, const double* X, double* F, hipStream_t st) {
  if (p.ninst > 1 && f.kind == FSIB_FORCE_CURVE_TENSION) {
    if (M <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_force_curve_inst, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, st, M, X, f.K,
                       (const int64_t*)p.inst_off, p.ninst, F);
    return hipGetLastError();
  }
  return launch_force(f, p.dim, M, X, F, st);  // the other laws index their mesh globally
}

template <typename T>
static hipError_t curve_group(const std::vector<Plan*>& ps, const fsib_force* f, const int64_t* M,
                              const double* const* X, hipStream_t st) {
  std::vector<PartLaunch<CurveArgs<T>>> v(ps.size());
  for (size_t g = 0; g < ps.size(); ++g) {
    const Plan& p = *ps[g];
    v[g].a = CurveArgs<T>{M[g], X[g], f[g].K, p.ninst > 1 ? (const int64_t*)p.inst_off : nullptr, p.ninst, p.F64,
                          (T*)p.S};
    v[g].nx = (M[g] + 255) / 256;
  }
  return launch_parts(
      v,
      [&](const PartLaunch<CurveArgs<T>>& L) {
        hipLaunchKernelGGL(k_curve_force_strengths<T>, dim3((unsigned)L.nx), dim3(256), 0, st, L.a);
        return hipGetLastError();
      },
      [&](const Parts<CurveArgs<T>>& fp, int64_t nwg, size_t, int) {
        hipLaunchKernelGGL(k_curve_force_strengths_parts<T>, dim3((unsigned)nwg), dim3(256), 0, st, fp);
        return hipGetLastError();
      });
}

// Force F and weighted strengths S of one plan in one pass where the law allows it (the closed curve,
// the surface), else the two launches of launch_force_plan and launch_weighted_strengths.
hipError_t launch_force_strengths(const Plan& p, const fsib_force& f, int64_t M, const double* X, double* F, void* S,
                                  hipStream_t st) {
  if (M <= 0) return hipSuccess;
  const unsigned nblk = (unsigned)((M + 255) / 256);
  if (f.kind == FSIB_FORCE_CURVE_TENSION && p.dim == 2) {
    const int64_t* off = p.ninst > 1 ? (const int64_t*)p.inst_off : nullptr;
    if (p.prec == FSIB_F64)
      hipLaunchKernelGGL(k_curve_force_strengths<double>, dim3(nblk), dim3(256), 0, st,
                         CurveArgs<double>{M, X, f.K, off, p.ninst, F, (double*)S});
    else
      hipLaunchKernelGGL(k_curve_force_strengths<float>, dim3(nblk), dim3(256), 0, st,
                         CurveArgs<float>{M, X, f.K, off, p.ninst, F, (float*)S});
    return hipGetLastError();
  }
  if (f.kind == FSIB_FORCE_SURFACE_TENSION && p.dim == 3)
    return launch_surface(SurfaceArgs{M, X, nullptr, 0.0, nullptr, f.K, f.tris, f.v2t_ptr, f.v2t_idx, F,
                                      p.prec == FSIB_F64 ? (double*)S : nullptr,
                                      p.prec == FSIB_F64 ? nullptr : (float*)S},
                          0, st);
  hipError_t e = launch_force_plan(p, f, M, X, F, st);
  if (e != hipSuccess) return e;
  return launch_weighted_strengths(p, f.kind, M, F, S, st);
}

// Xh = X + a U, then force and strengths at Xh as launch_force_strengths; the surface law does all of
// it in one pass, the other laws move the points first.
hipError_t launch_move_force_strengths(const Plan& p, const fsib_force& f, int64_t M, double* Xh, const double* X,
                                       const void* U, double a, double* F, void* S, hipStream_t st) {
  if (M <= 0) return hipSuccess;
  if (f.kind == FSIB_FORCE_SURFACE_TENSION && p.dim == 3)
    return launch_surface(SurfaceArgs{M, X, U, a, Xh, f.K, f.tris, f.v2t_ptr, f.v2t_idx, F,
                                      p.prec == FSIB_F64 ? (double*)S : nullptr,
                                      p.prec == FSIB_F64 ? nullptr : (float*)S},
                          p.prec == FSIB_F64 ? 1 : 2, st);
  hipError_t e = launch_axpy_positions(p, M, Xh, X, U, a, st);
  if (e != hipSuccess) return e;
  return launch_force_strengths(p, f, M, Xh, F, S, st);
}

// Force (into each plan's F64) and weighted strengths (into its S) for the plans of a group: one launch
// when every plan has the closed-curve law, else each plan's own pass.
hipError_t launch_force_strengths_group(const std::vector<Plan*>& ps, const fsib_force* f, const int64_t* M,
                                        const double* const* X, hipStream_t st) {
  bool curves = true;
  for (size_t g = 0; g < ps.size(); ++g) curves = curves && f[g].kind == FSIB_FORCE_CURVE_TENSION && ps[g]->dim == 2;
  if (curves)
    return ps[0]->prec == FSIB_F64 ? curve_group<double>(ps, f, M, X, st) : curve_group<float>(ps, f, M, X, st);
  for (size_t g = 0; g < ps.size(); ++g) {
    const hipError_t e = launch_force_strengths(*ps[g], f[g], M[g], X[g], ps[g]->F64, ps[g]->S, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_weighted_strengths(const Plan& p, int kind, int64_t M, const double* F, void* S, hipStream_t st) {
  const int64_t n = M * p.dim;
  if (n <= 0) return hipSuccess;
  if (p.ninst > 1 && kind == FSIB_FORCE_CURVE_TENSION) {
    const unsigned nb = (unsigned)((M + 255) / 256);
    if (p.prec == FSIB_F64)
      hipLaunchKernelGGL(k_strengths_inst<double>, dim3(nb), dim3(256), 0, st, M, p.dim, F,
                         (const int64_t*)p.inst_off, p.ninst, (double*)S);
    else
      hipLaunchKernelGGL(k_strengths_inst<float>, dim3(nb), dim3(256), 0, st, M, p.dim, F,
                         (const int64_t*)p.inst_off, p.ninst, (float*)S);
    return hipGetLastError();
  }
  const double w = force_weight(kind, M);
  const unsigned nblk = (unsigned)((n + 255) / 256);
  if (p.prec == FSIB_F64)
    hipLaunchKernelGGL(k_strengths<double>, dim3(nblk), dim3(256), 0, st, n, F, w, (double*)S);
  else
    hipLaunchKernelGGL(k_strengths<float>, dim3(nblk), dim3(256), 0, st, n, F, w, (float*)S);
  return hipGetLastError();
}

// ---- diagnostics: fixed-order FP64 reductions (deterministic) ----
constexpr int kDiagBlocks = 256;
constexpr int kDiagThreads = 256;
constexpr int kDiagSlots = 12;  // per block: 0..2 sum wF, 3 power, 4 E_K, 5 dissipation, 6 max |k.u|,
                                // 7 volume, 8 max |k||u|

__device__ __forceinline__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int o = kDiagThreads / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ double block_max(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int o = kDiagThreads / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

template <typename T>
__global__ __launch_bounds__(kDiagThreads) void k_diag_points(int64_t M, int dim, double w, const double* __restrict__ F,
                                                              const T* __restrict__ U, double* __restrict__ part) {
  __shared__ double sh[kDiagThreads];
  double s[3] = {0, 0, 0}, pw = 0;
  for (int64_t j = (int64_t)blockIdx.x * kDiagThreads + threadIdx.x; j < M; j += (int64_t)kDiagBlocks * kDiagThreads) {
    for (int a = 0; a < dim; ++a) {
      const double f = w * F[j * dim + a];
      s[a] += f;
      pw += f * (double)U[j * dim + a];
    }
  }
  for (int a = 0; a < 3; ++a) {
    const double r = block_sum(s[a], sh);
    if (threadIdx.x == 0) part[blockIdx.x * kDiagSlots + a] = r;
  }
  const double r = block_sum(pw, sh);
  if (threadIdx.x == 0) part[blockIdx.x * kDiagSlots + 3] = r;
}

template <typename T>
__global__ __launch_bounds__(kDiagThreads) void k_diag_modes(ModeGeo g, double rho, double mu,
                                                             const cplx<T>* __restrict__ u, double* __restrict__ part) {
  __shared__ double sh[kDiagThreads];
  const int64_t nm = g.Hx * g.N[1] * (g.dim == 3 ? g.N[2] : 1);
  double ek = 0, dis = 0, dv = 0, dn = 0;
  const double twopi_L = 6.283185307179586476925286766559 / g.L;
  for (int64_t idx = (int64_t)blockIdx.x * kDiagThreads + threadIdx.x; idx < nm;
       idx += (int64_t)kDiagBlocks * kDiagThreads) {
    const int64_t ix = idx % g.Hx;
    const int64_t iy = (idx / g.Hx) % g.N[1];
    const int64_t iz = g.dim == 3 ? idx / (g.Hx * g.N[1]) : 0;
    const double k[3] = {twopi_L * (double)ix, twopi_L * (double)mode_of(iy, g.N[1]),
                         g.dim == 3 ? twopi_L * (double)mode_of(iz, g.N[2]) : 0.0};
    // each stored mode with 0 < m_x < N_x/2 stands for itself and its conjugate partner
    const double wgt = (ix == 0 || 2 * ix == g.N[0]) ? 1.0 : 2.0;
    double uu = 0, kr = 0, ki = 0, k2 = 0;
    for (int a = 0; a < g.dim; ++a) {
      const cplx<T> v = u[a * nm + idx];
      uu += (double)v.x * v.x + (double)v.y * v.y;
      kr += k[a] * (double)v.x;
      ki += k[a] * (double)v.y;
      k2 += k[a] * k[a];
    }
    ek += wgt * uu;
    dis += wgt * k2 * uu;
    dv = fmax(dv, sqrt(kr * kr + ki * ki));
    dn = fmax(dn, sqrt(k2 * uu));
  }
  double r = block_sum(ek, sh);
  if (threadIdx.x == 0) part[blockIdx.x * kDiagSlots + 4] = r;
  r = block_sum(dis, sh);
  if (threadIdx.x == 0) part[blockIdx.x * kDiagSlots + 5] = r;
  r = block_max(dv, sh);
  if (threadIdx.x == 0) part[blockIdx.x * kDiagSlots + 6] = r;
  r = block_max(dn, sh);
  if (threadIdx.x == 0) part[blockIdx.x * kDiagSlots + 8] = r;
}

// enclosed area (2D shoelace over the closed curve) or volume (3D, (1/6) sum X_i . (X_j x X_k))
__global__ __launch_bounds__(kDiagThreads) void k_diag_volume(int dim, int64_t M, const double* __restrict__ X,
                                                              const int32_t* __restrict__ tris, int64_t ntris,
                                                              double* __restrict__ part) {
  __shared__ double sh[kDiagThreads];
  double v = 0;
  if (dim == 2) {
    for (int64_t j = (int64_t)blockIdx.x * kDiagThreads + threadIdx.x; j < M; j += (int64_t)kDiagBlocks * kDiagThreads) {
      const int64_t jp = j + 1 == M ? 0 : j + 1;
      v += 0.5 * (X[2 * j] * X[2 * jp + 1] - X[2 * jp] * X[2 * j + 1]);
    }
  } else if (tris) {
    for (int64_t t = (int64_t)blockIdx.x * kDiagThreads + threadIdx.x; t < ntris;
         t += (int64_t)kDiagBlocks * kDiagThreads) {
      const double* A = X + 3 * tris[3 * t];
      const double* B = X + 3 * tris[3 * t + 1];
      const double* C = X + 3 * tris[3 * t + 2];
      v += (A[0] * (B[1] * C[2] - B[2] * C[1]) + A[1] * (B[2] * C[0] - B[0] * C[2]) + A[2] * (B[0] * C[1] - B[1] * C[0])) /
           6.0;
    }
  }
  const double r = block_sum(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x * kDiagSlots + 7] = r;
}

template <typename T>
__global__ __launch_bounds__(kDiagThreads) void k_diag_final(int dim, double rho, double mu, double Ld,
                                                             const cplx<T>* __restrict__ u, int64_t nm,
                                                             const double* __restrict__ part, double* __restrict__ diag) {
  __shared__ double sh[kDiagThreads];
  double acc[9];
  for (int q = 0; q < 9; ++q) {
    const double v = threadIdx.x < kDiagBlocks ? part[threadIdx.x * kDiagSlots + q] : 0.0;
    acc[q] = (q == 6 || q == 8) ? block_max(v, sh) : block_sum(v, sh);
  }
  if (threadIdx.x == 0) {
    diag[0] = acc[0];
    diag[1] = acc[1];
    diag[2] = dim == 3 ? acc[2] : 0.0;
    for (int a = 0; a < 3; ++a) diag[3 + a] = a < dim ? (double)u[a * nm].x : 0.0;
    diag[6] = 0.5 * rho * Ld * acc[4];
    diag[7] = mu * Ld * acc[5];
    diag[8] = acc[3];
    diag[9] = acc[8] > 0 ? acc[6] / acc[8] : 0.0;
    diag[10] = acc[7];
  }
}

hipError_t launch_diag(const Plan& p, const fsib_fluid_params& prm, const fsib_force& f, int64_t M, const double* F,
                       const void* Uh, const void* uhat, const double* X, double* diag, hipStream_t st) {
  ModeGeo g;
  g.dim = p.dim;
  for (int a = 0; a < 3; ++a) g.N[a] = p.N[a];
  g.Hx = p.Hx;
  g.L = p.L;
  const double w = force_weight(f.kind, M);
  const double Ld = p.dim == 3 ? p.L * p.L * p.L : p.L * p.L;
  if (p.prec == FSIB_F64) {
    using T = double;
    hipLaunchKernelGGL(k_diag_points<T>, dim3(kDiagBlocks), dim3(kDiagThreads), 0, st, M, p.dim, w, F, (const T*)Uh,
                       p.part);
    hipLaunchKernelGGL(k_diag_modes<T>, dim3(kDiagBlocks), dim3(kDiagThreads), 0, st, g, prm.rho, prm.mu,
                       (const cplx<T>*)uhat, p.part);
  } else {
    using T = float;
    hipLaunchKernelGGL(k_diag_points<T>, dim3(kDiagBlocks), dim3(kDiagThreads), 0, st, M, p.dim, w, F, (const T*)Uh,
                       p.part);
    hipLaunchKernelGGL(k_diag_modes<T>, dim3(kDiagBlocks), dim3(kDiagThreads), 0, st, g, prm.rho, prm.mu,
                       (const cplx<T>*)uhat, p.part);
  }
  hipLaunchKernelGGL(k_diag_volume, dim3(kDiagBlocks), dim3(kDiagThreads), 0, st, p.dim, M, X,
                     f.ntris > 0 ? f.tris : nullptr, f.ntris, p.part);
  if (p.prec == FSIB_F64)
    hipLaunchKernelGGL(k_diag_final<double>, dim3(1), dim3(kDiagThreads), 0, st, p.dim, prm.rho, prm.mu, Ld,
                       (const cplx<double>*)uhat, p.modes_half(), (const double*)p.part, diag);
  else
    hipLaunchKernelGGL(k_diag_final<float>, dim3(1), dim3(kDiagThreads), 0, st, p.dim, prm.rho, prm.mu, Ld,
                       (const cplx<float>*)uhat, p.modes_half(), (const double*)p.part, diag);
  return hipGetLastError();
}

}  // namespace fsib
