// Plan (workspace + tables) of the FSIB library and the launchers of its kernels.
#pragma once

#include <algorithm>
#include <map>
#include <string>
#include <vector>

#include "common.hpp"
#include "../../include/fsib.h"

namespace fsib {

// Host-side numerics chosen at plan time (params.cpp).
double bessel_i0(double x);
double kb_transform(double a, double beta);  // int_{-1}^{1} I0(beta sqrt(1-z^2))/I0(beta) cos(a z) dz
int choose_width(double tol, int dim, double sigma);
double choose_beta(int w, double sigma);
int choose_degree(int w);
void fit_kernel_pieces(int w, double beta, int deg, double* coef /* (deg+1)*w */);
int64_t smooth_at_least(int64_t n, int64_t multiple);
int radix_plan(int n, int* radix);

struct Plan {
  // options
  int dim = 0;
  int64_t N[3] = {1, 1, 1};
  double L = 1.0;
  int prec = FSIB_F64;
  double tol = 1e-6;
  double sigma = 2.0;  // fine-grid oversampling
  int ntrans = 1;
  int64_t max_points = 0;
  int fluid = 0, ns = 0;
  int device = 0;
  int lds_max = 65536;  // LDS bytes one workgroup may allocate on this device
  int xcd_chunk_interp = 64;  // interpolation workgroups kept together per XCD (2048 sorted points)
  int xcd_chunk_spread = 16;  // spreading tiles kept together per XCD (0: plain numbering)
  int split = 512;            // candidates per part of a heavy spreading tile (set at creation: 256 up to 2^18 points)
  int split_alloc = 512;      // the split the work list and scratch were sized for (split >= it)
  // kernel
  int w = 0, deg = 0;
  double beta = 0.0;
  // grids
  int64_t nf[3] = {1, 1, 1};  // fine grid
  int64_t nd[3] = {1, 1, 1};  // dealiasing grid
  int64_t tb[3] = {1, 1, 1};  // tile (bin) size
  int64_t nt[3] = {1, 1, 1};  // tiles per axis
  int64_t nbins = 1;            // bins (tiles) of one instance
  int ninst = 1;                // independent instances sharing the plan (Stokes)
  int64_t nbt = 1;              // bins of all instances, nbins * ninst
  int64_t* inst_off = nullptr;  // device: ninst + 1 point offsets of the instances
  std::vector<int64_t> inst_off_h;  // host copy (empty until set)
  int64_t Hx = 1;             // half-spectrum length along x
  // device tables
  void* coef = nullptr;              // (deg+1)*w scalars of prec
  void* fac[3] = {nullptr, nullptr, nullptr};  // deconvolution factors per axis, N[a] scalars, FFT order
  std::map<int, void*> tw;           // twiddles per FFT length
  // point sort
  int* counts = nullptr;   // nbins+1
  bool counts_zero = false;  // host-side: counts are all zero (the last sort's scatter cleared them)
  int* offsets = nullptr;  // nbins+1
  int* pt_bin = nullptr;   // M
  int* pt_rank = nullptr;  // M
  int* s_idx = nullptr;    // M: original index of sorted point
  uint32_t* s_i0 = nullptr;  // M: packed first support cell (10 bits per axis)
  void* s_y = nullptr;     // M*dim prec: sub-cell position in [-1, 1]
  void* s_str = nullptr;   // strengths in sorted order: max(2 ntrans, dim) * M prec
  const void* sstr_src = nullptr;  // host-side: the real strengths the last sort placed in s_str (or none)
  int deterministic = 0;   // 1: each bin lists its points in ascending original index (k_bin_rank)
  int* det_key = nullptr;  // M: original index per claimed slot (deterministic plans only)
  int* flag = nullptr;     // non-finite position seen
  int* scan_part = nullptr;  // segment sums of the exclusive scans over bins
  uint8_t* rowmask = nullptr;  // nt[2] x nt[1]: a point's support reaches this block of x lines
  uint8_t* zmask = nullptr;    // nt[2]: some line of this block of z planes is reached
  // spreading work list (heavy tiles split into parts of at most `split` candidates)
  int64_t qn[3] = {0, 0, 0};   // bins before a tile, per axis, whose points can reach it
  int* tile_parts = nullptr;   // nbins
  int parts_split = 0;         // host-side: the split with which the last sort computed tile_parts (0: none)
  int* part_off = nullptr;     // nbins+1
  int* work = nullptr;         // 2 ints per part, work_blocks parts at most
  int* tile_slot = nullptr;    // nbins
  int* slot_ctr = nullptr;     // [0]: scratch slots claimed, [1]: split tiles listed
  int* split_list = nullptr;   // the split tiles (at most split_slots / 2 + 1)
  void* split_scratch = nullptr;
  int64_t work_blocks = 0;     // bound on the number of parts
  int64_t split_slots = 0;     // bound on the partial tiles of split tiles (per transform)
  // grids / FFT buffers
  void* grid = nullptr;
  void* B1 = nullptr;
  void* B2 = nullptr;
  // FSIB workspace
  double* Xh = nullptr;    // M*dim
  double* F64 = nullptr;   // M*dim
  void* S = nullptr;       // M*dim prec
  void* Uh = nullptr;      // M*dim prec
  void* fhat = nullptr;    // dim half spectra
  void* uhat_mid = nullptr;
  void* pihat = nullptr;   // dealiased products, nprod half spectra
  void* D1 = nullptr;      // dealiasing FFT buffers
  void* D2 = nullptr;
  void* prod = nullptr;    // nprod half spectra in x on the dealiasing grid in y, z
  double* part = nullptr;  // reduction partials
  int npart = 0;
  int64_t ws_bytes = 0;
  // Navier-Stokes steps: a second stream (default priority) for the point side of each half step
  // and the events that fork it from and join it to the caller's stream
  hipStream_t aux = nullptr;
  int overlap = 1;
  int interp_points = 4;  // points per interpolation wavefront (4 measured faster than 8 and 16)
  int spread_threads = 0; // threads per spreading tile (0: the default of the dimension and precision)
  int nl_stages = 0;      // FFT stages of the fused products x pass on 192-point lines (0: automatic)
  hipEvent_t fj[4] = {nullptr, nullptr, nullptr, nullptr};
  // optional timing of one kernel class with HIP events on the launch stream
  int prof_class = -1;
  std::vector<hipEvent_t> prof_ev;  // start/stop pairs
  mutable int prof_used = 0;
  mutable double prof_bytes = 0.0;

  int64_t fine_cells() const { return nf[0] * nf[1] * nf[2]; }
  int64_t modes_full() const { return N[0] * N[1] * N[2]; }
  int64_t modes_half() const { return Hx * N[1] * N[2]; }
  int64_t dealias_cells() const { return nd[0] * nd[1] * nd[2]; }
  int nprod() const { return dim == 3 ? 6 : 3; }
  size_t real_size() const { return prec == FSIB_F64 ? 8 : 4; }
};

// ---- launches over the plans of a group ----
// One part of such a launch: the arguments, grid, workgroup size and dynamic LDS its kernel would
// get in a launch of its own.
template <class A>
struct PartLaunch {
  A a;
  int64_t nx = 0, ny = 1;
  int threads = 256;
  size_t lds = 0;
};

// One launch for all parts when there are several that share a workgroup size (`fused(parts,
// workgroups, lds, threads)`), else a launch per part (`one(part)`); parts with an empty grid are left
// out.
template <class A, class One, class Fused>
hipError_t launch_parts(const std::vector<PartLaunch<A>>& v, One one, Fused fused) {
  static_assert(sizeof(Parts<A>) <= 4096, "kernel arguments of a launch over parts");
  std::vector<const PartLaunch<A>*> live;
  for (const auto& q : v)
    if (q.nx * q.ny > 0) live.push_back(&q);
  if (live.empty()) return hipSuccess;
  // smallest grid first: workgroups are dispatched in order, and a part's long-running workgroups
  // (the crowded tiles of spreading) then start before the many short ones of the largest grid
  std::stable_sort(live.begin(), live.end(),
                   [](const PartLaunch<A>* a, const PartLaunch<A>* b) { return a->nx * a->ny < b->nx * b->ny; });
  bool same = live.size() <= (size_t)kMaxParts;
  for (const auto* q : live) same = same && q->threads == live[0]->threads;
  if (live.size() == 1 || !same) {
    for (const auto* q : live) {
      const hipError_t e = one(*q);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  Parts<A> f;
  f.n = (int)live.size();
  int64_t s = 0;
  size_t lds = 0;
  for (int g = 0; g < f.n; ++g) {
    f.a[g] = live[g]->a;
    f.nx[g] = (uint32_t)live[g]->nx;
    f.ny[g] = (uint32_t)live[g]->ny;
    f.start[g] = (uint32_t)s;
    s += (live[g]->nx * live[g]->ny + kXcds - 1) / kXcds * kXcds;
    lds = lds > live[g]->lds ? lds : live[g]->lds;
  }
  if (s >= ((int64_t)1 << 32) - kXcds) return hipErrorInvalidConfiguration;
  for (int g = f.n; g <= kMaxParts; ++g) f.start[g] = (uint32_t)s;
  return fused(f, s, lds, live[0]->threads);
}

// ---- launchers (all asynchronous on `st`) ----
// points.hip
// str (nullable): real strengths (dim per point, plan precision) that the spreading after this sort
// will take; the scatter then also places them in sorted order
hipError_t launch_sort_points(Plan& p, int64_t M, const double* X, hipStream_t st, const void* str = nullptr);
hipError_t launch_spectral_scale(const Plan& p, int layout, int axis, double scale, const void* in, void* out,
                                 hipStream_t st);  // layout 0: ntrans full spectra; 1: dim half spectra
hipError_t launch_grad_combine(const Plan& p, int64_t M, int kind, const void* u, const void* v, const void* u2,
                               const void* v2, double scale, double* gX, int axis, hipStream_t st);
hipError_t launch_axpy_positions(const Plan& p, int64_t M, double* Y, const double* X, const void* U,
                                 double a, hipStream_t st);  // Y = X + a*U
hipError_t launch_fill_zero(void* ptr, int64_t bytes, hipStream_t st);
// exclusive, n+1 outputs; seg_sum: scan_segments(n) ints; clear (nullable): three ints zeroed
hipError_t launch_scan(int64_t n, const int* counts, int* offsets, int* seg_sum, hipStream_t st,
                       int* clear = nullptr);
int64_t scan_segments(int64_t n);
// the scan of the tiles' part counts `counts`, whose final pass also writes the spreading work list
// (points.hip); per plan of a group in one launch per pass
struct FillWorkArgs;
hipError_t launch_scan_fill_work(int64_t n, const int* counts, int* offsets, int* seg_sum, const FillWorkArgs& f,
                                 hipStream_t st);
hipError_t launch_scan_fill_work_group(const std::vector<int64_t>& n, const std::vector<const int*>& counts,
                                       const std::vector<int*>& offsets, const std::vector<int*>& seg_sum,
                                       const std::vector<FillWorkArgs>& f, hipStream_t st);
hipError_t launch_row_masks(Plan& p, int64_t M, hipStream_t st);  // from the bin counts of M points
// the same stages for the plans of a group, each one launch over all plans where their workgroup
// sizes agree (plan g: M[g] points, its operands at index g)
hipError_t launch_sort_points_group(const std::vector<Plan*>& ps, const int64_t* M, const double* const* X,
                                    hipStream_t st, const void* const* str = nullptr);
hipError_t launch_axpy_positions_group(const std::vector<Plan*>& ps, const int64_t* M, double* const* Y,
                                       const double* const* X, const void* const* U, const double* a,
                                       hipStream_t st);
hipError_t launch_fill_zero_group(const std::vector<void*>& ptr, const std::vector<int64_t>& bytes, hipStream_t st);
hipError_t launch_scan_group(const std::vector<int64_t>& n, const std::vector<const int*>& counts,
                             const std::vector<int*>& offsets, const std::vector<int*>& seg_sum, hipStream_t st);
hipError_t launch_spread_group(const std::vector<Plan*>& ps, const int64_t* M, const void* const* str,
                               hipStream_t st);  // real strengths with dim components
// position updates done by an interpolation pass over a group: out[g] = in[g] + a[g] U[g] (U as stored)
struct GroupMove {
  double* const* out;
  const double* const* in;
  const double* a;
};
hipError_t launch_interp_group(const std::vector<Plan*>& ps, const int64_t* M, void* const* out, hipStream_t st,
                               const GroupMove* mv = nullptr);
hipError_t launch_force_strengths_group(const std::vector<Plan*>& ps, const fsib_force* f, const int64_t* M,
                                        const double* const* X, hipStream_t st);  // into each plan's F64, S
hipError_t launch_fluid_stokes_group(const std::vector<Plan*>& ps, const fsib_fluid_params* prm,
                                     void* const* uhat, hipStream_t st);  // from each plan's fhat
// FFT passes of several plans: the operands of one launch_fft_c2c call (x passes: outer = real rows,
// r2c keeps nout entries with fac_out, c2r reads nin with fac_in)
struct FftCall {
  const Plan* p;
  const void* in;
  void* out;
  int n, sign;
  int64_t inner, outer;
  int nin, pin, nout, pout;
  const void* fac_in;
  const void* fac_out;
  double scale;
  PassMasks mk;
};
hipError_t launch_fft_c2c_group(const std::vector<FftCall>& calls, hipStream_t st);
hipError_t launch_fft_x_group(const std::vector<FftCall>& calls, bool r2c, hipStream_t st);
// spread_interp.hip
hipError_t launch_spread(Plan& p, int64_t M, const void* strengths, int real_comps, hipStream_t st);
// move (real strengths, nullable): positions also advanced, move += move_a * out (as stored)
hipError_t launch_interp(Plan& p, int64_t M, void* out, int real_comps, hipStream_t st, double* move = nullptr,
                         double move_a = 0);
// fft.hip
hipError_t launch_fft_c2c(const Plan& p, const void* in, void* out, int n, int sign, int64_t inner,
                          int64_t outer, int nin, int pin, int nout, int pout, const void* fac_in,
                          const void* fac_out, double scale, hipStream_t st, const PassMasks& mk = PassMasks());
hipError_t launch_fft_r2c_x(const Plan& p, const void* in, void* out, int n, int64_t rows, int nout,
                            const void* fac_out, double scale, hipStream_t st, const PassMasks& mk = PassMasks());
hipError_t launch_fft_c2r_x(const Plan& p, const void* in, void* out, int n, int64_t rows, int nin,
                            const void* fac_in, double scale, hipStream_t st, const PassMasks& mk = PassMasks());
// fluid.hip
// nonlinear.hip; stages (2 or 3) picks the kernel of 192-point lines, other lengths have one
hipError_t launch_nl_xpass(const Plan& p, const void* in, void* out, int stages, hipStream_t st);
bool fft_line_fits(const Plan& p, int n);  // fft.hip
bool nl_line_fits(const Plan& p, int n);   // nonlinear.hip
// products_fluid.hip: the forward z pass of the products (from p.D1) fused with the Navier-Stokes
// update, for 3D plans with 128 modes and 192 dealiasing points along z
bool products_z_fluid_fits(const Plan& p);
hipError_t launch_products_z_fluid(const Plan& p, int mode, const fsib_fluid_params& prm, const void* fhat,
                                   const void* uin, void* uout, hipStream_t st);
hipError_t launch_fluid_update(const Plan& p, int mode, const fsib_fluid_params& prm, const void* fhat,
                               const void* uin, void* uout, hipStream_t st);
hipError_t launch_force(const fsib_force& f, int dim, int64_t M, const double* X, double* F,
                        hipStream_t st);
hipError_t launch_pressure(const Plan& p, int ns, double rho, const void* fhat, void* phat, hipStream_t st);
hipError_t launch_spring_stiffness(int64_t M, const double* X0, const int32_t* tris, const int32_t* v2t_ptr,
                                   const int32_t* v2t_idx, const int32_t* nptr, const int32_t* nbr, double* kij,
                                   int* missing, hipStream_t st);
hipError_t launch_force_plan(const Plan& p, const fsib_force& f, int64_t M, const double* X, double* F, hipStream_t st);
hipError_t launch_force_jvp(const fsib_force& f, int dim, int64_t M, const double* X, const double* V, double* out,
                            hipStream_t st);
hipError_t launch_force_strengths(const Plan& p, const fsib_force& f, int64_t M, const double* X, double* F, void* S,
                                  hipStream_t st);  // F and S = w F in one pass where the law allows
// Xh = X + a U (U in the plan precision), then F and S at Xh (one pass for the surface law)
hipError_t launch_move_force_strengths(const Plan& p, const fsib_force& f, int64_t M, double* Xh, const double* X,
                                       const void* U, double a, double* F, void* S, hipStream_t st);
hipError_t launch_weighted_strengths(const Plan& p, int kind, int64_t M, const double* F, void* S,
                                     hipStream_t st);
hipError_t launch_diag(const Plan& p, const fsib_fluid_params& prm, const fsib_force& f, int64_t M,
                       const double* F, const void* Uh, const void* uhat, const double* X, double* diag,
                       hipStream_t st);

// api.cpp: the last-error message of this thread, and type-1 through a caller-given device workspace
fsib_status report(fsib_status s, const char* msg);
fsib_status spread_in_workspace(fsib_plan plan, int device, int64_t M, const double* X, const void* c, void* fhat,
                                double scale, void* stream, void* ws, int64_t ws_bytes);

// Kernel classes that fsib_plan_profile can time (values of fsib_prof_class).
enum { PROF_FFT_STRIDED = 1, PROF_SPREAD = 2, PROF_INTERP = 3, PROF_FFT_X = 4, PROF_NL_X = 5 };

inline bool prof_on(const Plan& p, int cls) {
  return p.prof_class == cls && 2 * (size_t)p.prof_used + 1 < p.prof_ev.size();
}
inline void prof_start(const Plan& p, hipStream_t st) { (void)hipEventRecord(p.prof_ev[2 * p.prof_used], st); }
inline void prof_stop(const Plan& p, double bytes, hipStream_t st) {
  (void)hipEventRecord(p.prof_ev[2 * p.prof_used + 1], st);
  ++p.prof_used;
  p.prof_bytes += bytes;
}

// fluid update modes
enum { FLUID_STOKES = 0, FLUID_NS_HALF = 1, FLUID_NS_FULL = 2 };

}  // namespace fsib
