// C ABI of the FSIB library: plan construction and the orchestration of the kernels for the
// nonuniform transforms (App. A), the FSIB coupling (Sec. 3.1), the fluid update and Alg. 1.
#include <cstdlib>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <set>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "plan.hpp"

struct fsib_plan_s {
  fsib::Plan p;
};

namespace {

thread_local std::string g_last_error;

fsib_status fail(fsib_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

#define FSIB_HIP(call)                                                                                  \
  do {                                                                                                  \
    hipError_t e_ = (call);                                                                             \
    if (e_ != hipSuccess)                                                                               \
      return fail(FSIB_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_));                     \
  } while (0)

#define FSIB_TRY(call)                 \
  do {                                 \
    fsib_status s_ = (call);           \
    if (s_ != FSIB_OK) return s_;      \
  } while (0)

using fsib::Plan;


int64_t ceil_half(int64_t n) { return (n + 1) / 2; }

struct Alloc {
  Plan& p;
  fsib_status status = FSIB_OK;
  template <typename P>
  void get(P*& ptr, int64_t bytes) {
    if (status != FSIB_OK) return;
    if (bytes <= 0) bytes = 256;
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, (size_t)bytes);
    if (e != hipSuccess) {
      status = FSIB_ERR_OOM;
      g_last_error = std::string("hipMalloc of ") + std::to_string(bytes) + " bytes: " + hipGetErrorString(e);
      return;
    }
    ptr = (P*)q;
    p.ws_bytes += bytes;
  }
};

void free_plan(Plan& p) {
  auto fr = [](void* q) {
    if (q) (void)hipFree(q);
  };
  for (hipEvent_t e : p.prof_ev) (void)hipEventDestroy(e);
  p.prof_ev.clear();
  for (hipEvent_t& e : p.fj)
    if (e) {
      (void)hipEventDestroy(e);
      e = nullptr;
    }
  if (p.aux) {
    (void)hipStreamDestroy(p.aux);
    p.aux = nullptr;
  }
  fr(p.coef);
  for (int a = 0; a < 3; ++a) fr(p.fac[a]);
  for (auto& kv : p.tw) fr(kv.second);
  p.tw.clear();
  fr(p.counts);
  fr(p.offsets);
  fr(p.inst_off);
  fr(p.pt_bin);
  fr(p.pt_rank);
  fr(p.det_key);
  fr(p.s_idx);
  fr(p.s_i0);
  fr(p.s_y);
  fr(p.s_str);
  fr(p.flag);
  fr(p.scan_part);
  fr(p.rowmask);
  fr(p.zmask);
  fr(p.tile_parts);
  fr(p.part_off);
  fr(p.work);
  fr(p.tile_slot);
  fr(p.slot_ctr);
  fr(p.split_list);
  fr(p.split_scratch);
  fr(p.grid);
  fr(p.B1);
  fr(p.B2);
  fr(p.Xh);
  fr(p.F64);
  fr(p.S);
  fr(p.Uh);
  fr(p.fhat);
  fr(p.uhat_mid);
  fr(p.pihat);
  fr(p.D1);
  fr(p.D2);
  fr(p.prod);
  fr(p.part);
}

// host -> device copy of a double table converted to the plan precision
fsib_status upload(const Plan& p, void* dst, const std::vector<double>& v) {
  if (p.prec == FSIB_F64) {
    FSIB_HIP(hipMemcpy(dst, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice));
  } else {
    std::vector<float> f(v.begin(), v.end());
    FSIB_HIP(hipMemcpy(dst, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice));
  }
  return FSIB_OK;
}

// Oversampling of a plan: upsampfac 2.0, 1.5 or 1.25 as asked; 0 picks 1.5 for 3D plans whose point
// count is small against the mode count (max_points <= N^3 / 20), where the FFT passes over the fine
// grid outweigh the wider kernel, in FP64 at tol >= 1e-6 (128^3 modes, 4e4 points, tol 1e-5: 1.247 ms
// per Navier-Stokes step at 1.5 with w = 8, 1.345 ms at 1.25 with w = 10, more at 2.0) and in FP32 at
// tol >= 1e-4; 2.0 otherwise.
static double plan_sigma(const fsib_plan_opts* o) {
  if (o->upsampfac == 1.25 || o->upsampfac == 1.5 || o->upsampfac == 2.0) return o->upsampfac;
  const double modes = (double)o->n_modes[0] * (double)o->n_modes[1] * (o->dim == 3 ? (double)o->n_modes[2] : 1.0);
  const bool small_m = 20.0 * (double)o->max_points <= modes;
  if (o->dim == 3 && small_m) {
    if (o->prec == FSIB_F64 && o->tol >= 1e-6) return 1.5;
    // FP32 rounding lifted ~8x by the deconvolution at 1.5 puts multi-step results near 3e-5 of the
    // exact sums: 1.5 only where that is within the tolerance
    if (o->prec == FSIB_F32 && o->tol >= 1e-4) return 1.5;
  }
  return 2.0;
}

fsib_status validate_opts(const fsib_plan_opts* o) {
  if (!o) return fail(FSIB_ERR_ARG, "opts is NULL");
  if (o->dim != 2 && o->dim != 3) return fail(FSIB_ERR_ARG, "dim must be 2 or 3");
  for (int a = 0; a < o->dim; ++a)
    if (o->n_modes[a] < 2 || o->n_modes[a] > 4096) return fail(FSIB_ERR_ARG, "n_modes must be in [2, 4096]");
  if (!(o->L > 0) || !std::isfinite(o->L)) return fail(FSIB_ERR_ARG, "L must be positive and finite");
  if (o->prec != FSIB_F64 && o->prec != FSIB_F32) return fail(FSIB_ERR_ARG, "prec must be FSIB_F64 or FSIB_F32");
  if (!(o->upsampfac == 0.0 || o->upsampfac == 2.0 || o->upsampfac == 1.5 || o->upsampfac == 1.25))
    return fail(FSIB_ERR_ARG, "upsampfac must be 0, 2.0, 1.5 or 1.25");
  if (o->ntrans < 1 || o->ntrans > 65535) return fail(FSIB_ERR_ARG, "ntrans must be in [1, 65535]");
  if (o->max_points < 0 || o->max_points > (int64_t)1 << 30) return fail(FSIB_ERR_ARG, "max_points out of range");
  if (!std::isfinite(o->tol) || o->tol > 0.1) return fail(FSIB_ERR_TOL, "tol must be <= 0.1");
  if (o->prec == FSIB_F64 && !(o->tol >= 1e-14)) return fail(FSIB_ERR_TOL, "FP64 plans reach tol >= 1e-14");
  if (o->prec == FSIB_F32 && !(o->tol >= 1e-6)) return fail(FSIB_ERR_TOL, "FP32 plans reach tol >= 1e-6");
  if (o->navier_stokes && !o->fluid) return fail(FSIB_ERR_ARG, "navier_stokes needs fluid = 1");
  if (o->deterministic != 0 && o->deterministic != 1) return fail(FSIB_ERR_ARG, "deterministic must be 0 or 1");
  if (o->ninst < 0 || o->ninst > 4096) return fail(FSIB_ERR_ARG, "ninst must be in [0, 4096]");
  if (o->ninst > 1 && (!o->fluid || o->navier_stokes || o->ntrans != 1))
    return fail(FSIB_ERR_ARG, "ninst > 1 needs fluid = 1, navier_stokes = 0 and ntrans = 1");
  // at oversampling 1.25 the kernel transform falls by up to ~100x across the retained modes, and the
  // deconvolution lifts FP32 rounding of the grid by as much: FP32 low-memory plans stop at 1e-3
  if (plan_sigma(o) == 1.25 && o->prec == FSIB_F32 && !(o->tol >= 1e-3))
    return fail(FSIB_ERR_TOL, "FP32 plans with upsampfac 1.25 reach tol >= 1e-3");
  // at 1.5 the transform falls by about 10x across the retained modes (w = 8): FP32 stops at 1e-5
  if (plan_sigma(o) == 1.5 && o->prec == FSIB_F32 && !(o->tol >= 1e-5))
    return fail(FSIB_ERR_TOL, "FP32 plans with upsampfac 1.5 reach tol >= 1e-5");
  if (fsib::choose_width(o->tol, o->dim, plan_sigma(o)) > fsib::kMaxW)
    return fail(FSIB_ERR_TOL, "tol is out of reach of the kernel widths available at this oversampling");
  return FSIB_OK;
}

fsib_status build_plan(Plan& p, const fsib_plan_opts* o) {
  p.dim = o->dim;
  for (int a = 0; a < 3; ++a) p.N[a] = a < o->dim ? o->n_modes[a] : 1;
  p.L = o->L;
  p.prec = o->prec;
  p.tol = o->tol;
  p.ntrans = o->ntrans;
  p.max_points = o->max_points;
  p.fluid = o->fluid ? 1 : 0;
  p.ns = o->navier_stokes ? 1 : 0;
  p.deterministic = o->deterministic ? 1 : 0;
  FSIB_HIP(hipGetDevice(&p.device));
  FSIB_HIP(hipDeviceGetAttribute(&p.lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, p.device));
  // workgroup-to-XCD run lengths (tuning knobs; the defaults are the measured best)
  // (the environment may replace them at creation; values outside [0, 4096] are ignored)
  auto env_chunk = [](const char* name, int& v) {
    if (const char* e = std::getenv(name)) {
      const int c = std::atoi(e);
      if (c >= 0 && c <= 4096) v = c;
    }
  };
  env_chunk("FSIB_XCD_CHUNK_INTERP", p.xcd_chunk_interp);
  env_chunk("FSIB_XCD_CHUNK_SPREAD", p.xcd_chunk_spread);
  // kernel (App. A.3): width from tol, Kaiser-Bessel shape, polynomial degree
  p.sigma = plan_sigma(o);
  p.w = fsib::choose_width(p.tol, p.dim, p.sigma);
  if (p.w > fsib::kMaxW)
    return fail(FSIB_ERR_TOL, "tol is out of reach of the kernel widths available at this oversampling");
  p.beta = fsib::choose_beta(p.w, p.sigma);
  p.deg = fsib::choose_degree(p.w);
  // fine grid and tiles: n_f >= sigma N and >= 2w, 2^a 3^b 5^c, a multiple of the tile
  // spreading tiles: 16 cells along x (one register row per thread), <= 1024 cells, <= 256 rows
  const int64_t tile3[3] = {16, 8, 8}, tile2[3] = {16, 16, 1};
  for (int a = 0; a < 3; ++a) {
    if (a >= p.dim) {
      p.nf[a] = p.tb[a] = p.nt[a] = 1;
      continue;
    }
    const int64_t tb = p.dim == 3 ? tile3[a] : tile2[a];
    int64_t need = p.sigma == 2.0 ? 2 * p.N[a] : (p.sigma == 1.5 ? (3 * p.N[a] + 1) / 2 : (5 * p.N[a] + 3) / 4);  // ceil(sigma N)
    if (need < 2 * p.w) need = 2 * p.w;
    if (need < tb) need = tb;
    p.nf[a] = fsib::smooth_at_least(need, tb);
    p.tb[a] = tb;
    p.nt[a] = p.nf[a] / tb;
  }
  if (p.dim == 3 && (p.nf[0] > 1024 || p.nf[1] > 1024 || p.nf[2] > 1024))
    return fail(FSIB_ERR_ARG, "3D fine grid above 1024 per axis (n_modes above 512) is not supported");
  if (p.dim == 2 && (p.nf[0] > 65535 || p.nf[1] > 65535)) return fail(FSIB_ERR_ARG, "2D fine grid too large");
  p.nbins = p.nt[0] * p.nt[1] * p.nt[2];
  p.ninst = o->ninst > 1 ? o->ninst : 1;
  p.nbt = p.nbins * p.ninst;
  p.Hx = p.N[0] / 2 + 1;
  if (p.ns) {
    for (int a = 0; a < 3; ++a) {
      if (a >= p.dim) {
        p.nd[a] = 1;
        continue;
      }
      const int64_t n = p.N[a];
      // Ntilde >= 3N/2 (Sec. 3.1) for the Nyquist-free field; odd N: > 3(N-1)/2
      const int64_t need = n % 2 == 0 ? (3 * n) / 2 : (3 * (n - 1)) / 2 + 1;
      p.nd[a] = fsib::smooth_at_least(need, 2);
    }
  }
  // FFT lengths must have a radix plan
  std::set<int> lengths;
  for (int a = 0; a < p.dim; ++a) {
    lengths.insert((int)p.nf[a]);
    if (p.ns) lengths.insert((int)p.nd[a]);
  }
  for (int n : lengths) {
    int r[fsib::kMaxStages];
    if (fsib::radix_plan(n, r) == 0) return fail(FSIB_ERR_ARG, "no FFT radix plan for length " + std::to_string(n));
    // one FFT line must fit one workgroup's threads and LDS on this device
    if (!fsib::fft_line_fits(p, n))
      return fail(FSIB_ERR_ARG, "FFT length " + std::to_string(n) + " exceeds the LDS budget of one workgroup (" +
                                    std::to_string(p.lds_max) + " bytes) or its thread limit");
  }
  if (p.ns && !fsib::nl_line_fits(p, (int)p.nd[0]))
    return fail(FSIB_ERR_ARG, "dealiasing length " + std::to_string(p.nd[0]) +
                                  " exceeds one workgroup of the nonlinear term's x pass");

  const int64_t rs = (int64_t)p.real_size();
  const int64_t cs = 2 * rs;
  const int64_t Mx = p.max_points > 0 ? p.max_points : 1;
  const int64_t d = p.dim;
  const int64_t nfc = p.fine_cells();
  Alloc A{p};
  A.get(p.coef, (int64_t)(p.deg + 1) * p.w * rs);
  for (int a = 0; a < p.dim; ++a) A.get(p.fac[a], p.N[a] * rs);
  for (int n : lengths) {
    void* t = nullptr;
    A.get(t, (int64_t)n * cs);
    if (t) p.tw[n] = t;
  }
  A.get(p.counts, (p.nbt + 1) * 4);
  A.get(p.offsets, (p.nbt + 1) * 4);
  A.get(p.inst_off, (int64_t)(p.ninst + 1) * 8);
  A.get(p.pt_bin, Mx * 4);
  A.get(p.pt_rank, Mx * 4);
  if (p.deterministic) A.get(p.det_key, Mx * 4);
  A.get(p.s_idx, Mx * 4);
  A.get(p.s_i0, Mx * 4);
  A.get(p.s_y, Mx * d * rs);
  A.get(p.s_str, Mx * (2 * p.ntrans > d ? 2 * p.ntrans : d) * rs);
  A.get(p.flag, 256);
  A.get(p.scan_part, fsib::scan_segments(p.nbt) * 4);
  A.get(p.rowmask, p.nt[1] * p.nt[2] * (p.dim == 2 ? p.ninst : 1));  // 2D: one block per instance
  A.get(p.zmask, p.nt[2]);
  // spreading work list: part bound = tiles + visits / split, visits <= M * prod(q + 1)
  {
    int64_t reach = 1;
    for (int a = 0; a < p.dim; ++a) {
      int64_t q = (p.w - 1 + p.tb[a] - 1) / p.tb[a];
      if (q > p.nt[a] - 1) q = p.nt[a] - 1;
      p.qn[a] = q;
      reach *= q + 1;
    }
    const int64_t visits = Mx * reach;
    // crowded tiles split into parts of 256 candidates (measured best for the FP64 step of the 128^3
    // surface: 1.099 ms against 1.104 with 192 and 1.108 with 128), 128 in FP32 Navier-Stokes plans
    // (0.792 against 0.799 ms with 256: at oversampling 2 the tiles are smaller against the kernel);
    // plans of many points keep 512, which halves the bound on the partial-tile scratch
    p.split = Mx <= ((int64_t)1 << 18) ? (p.ns && p.prec == FSIB_F32 ? 128 : 256) : 512;
    // FSIB_SPREAD_SPLIT overrides it at creation (clamped to [64, 2^20]); the tuning knob can only
    // raise it
    if (const char* e = std::getenv("FSIB_SPREAD_SPLIT")) {
      const int v = std::atoi(e);
      p.split = v < 64 ? 64 : (v > (1 << 20) ? (1 << 20) : v);
    }
    p.split_alloc = p.split;
    p.work_blocks = p.nbt + visits / p.split + 1;
    p.split_slots = 2 * visits / p.split + 2;
    const int64_t nch_bytes = 2 * rs > d * rs ? 2 * rs : d * rs;  // complex or dim real channels
    const int64_t tr = p.ntrans > 1 ? p.ntrans : 1;
    A.get(p.tile_parts, p.nbt * 4);
    A.get(p.part_off, (p.nbt + 1) * 4);
    A.get(p.work, p.work_blocks * 8);
    A.get(p.tile_slot, p.nbt * 4);
    A.get(p.slot_ctr, 256);
    A.get(p.split_list, (p.split_slots / 2 + 1) * 4);
    A.get(p.split_scratch, tr * p.split_slots * 1024 * nch_bytes);
  }
  // grid and FFT buffers: complex transforms (ntrans) and, for fluid plans, dim real fields
  int64_t grid_b = (int64_t)p.ntrans * nfc * cs;
  int64_t b1 = p.dim == 3 ? (int64_t)p.ntrans * p.nf[2] * p.nf[1] * p.N[0] * cs : (int64_t)p.ntrans * p.nf[1] * p.N[0] * cs;
  int64_t b2 = p.dim == 3 ? (int64_t)p.ntrans * p.nf[2] * p.N[1] * p.N[0] * cs : 0;
  if (p.fluid) {
    const int64_t dn = d * p.ninst;  // real fields of all instances
    const int64_t gr = dn * nfc * rs;
    const int64_t r1 = p.dim == 3 ? dn * p.nf[2] * p.nf[1] * p.Hx * cs : dn * p.nf[1] * p.Hx * cs;
    const int64_t r2 = p.dim == 3 ? dn * p.nf[2] * p.N[1] * p.Hx * cs : 0;
    grid_b = grid_b > gr ? grid_b : gr;
    b1 = b1 > r1 ? b1 : r1;
    b2 = b2 > r2 ? b2 : r2;
  }
  A.get(p.grid, grid_b);
  A.get(p.B1, b1);
  A.get(p.B2, b2);
  if (p.fluid) {
    A.get(p.Xh, Mx * d * 8);
    A.get(p.F64, Mx * d * 8);
    A.get(p.S, Mx * d * rs);
    A.get(p.Uh, Mx * d * rs);
    A.get(p.fhat, d * p.ninst * p.modes_half() * cs);
    A.get(p.uhat_mid, d * p.ninst * p.modes_half() * cs);
    A.get(p.part, 256 * 12 * 8);
  }
  if (p.ns) {
    const int64_t nc = p.nprod() > d ? p.nprod() : d;
    A.get(p.pihat, p.nprod() * p.modes_half() * cs);
    A.get(p.D1, p.dim == 3 ? nc * p.nd[2] * p.N[1] * p.Hx * cs : 0);
    A.get(p.D2, p.dim == 3 ? nc * p.nd[2] * p.nd[1] * p.Hx * cs : nc * p.nd[1] * p.Hx * cs);
    A.get(p.prod, p.dim == 3 ? p.nprod() * p.nd[2] * p.nd[1] * p.Hx * cs : p.nprod() * p.nd[1] * p.Hx * cs);
  }
  if (A.status != FSIB_OK) return A.status;
  if (p.ns) {
    FSIB_HIP(hipStreamCreateWithFlags(&p.aux, hipStreamNonBlocking));
    for (hipEvent_t& e : p.fj) FSIB_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }

  // tables
  std::vector<double> coef((size_t)(p.deg + 1) * p.w);
  fsib::fit_kernel_pieces(p.w, p.beta, p.deg, coef.data());
  FSIB_TRY(upload(p, p.coef, coef));
  for (int a = 0; a < p.dim; ++a) {
    // deconvolution: the fine-grid FFT of the spread carries (w/2) Ghat(pi m w / n_f) per axis
    std::vector<double> f((size_t)p.N[a]);
    for (int64_t i = 0; i < p.N[a]; ++i) {
      const int64_t m = i < ceil_half(p.N[a]) ? i : i - p.N[a];
      f[(size_t)i] = 2.0 / (p.w * fsib::kb_transform(M_PI * (double)m * p.w / (double)p.nf[a], p.beta));
    }
    FSIB_TRY(upload(p, p.fac[a], f));
  }
  for (auto& kv : p.tw) {
    const int n = kv.first;
    std::vector<double> t(2 * (size_t)n);
    for (int i = 0; i < n; ++i) {
      const long double ang = -2.0L * (long double)M_PI * (long double)i / (long double)n;
      t[2 * (size_t)i] = (double)cosl(ang);
      t[2 * (size_t)i + 1] = (double)sinl(ang);
    }
    FSIB_TRY(upload(p, kv.second, t));
  }
  FSIB_HIP(hipMemset(p.flag, 0, 256));
  FSIB_HIP(hipDeviceSynchronize());
  return FSIB_OK;
}

hipStream_t S(void* s) { return (hipStream_t)s; }

// Occupancy masks of the fine grid for the passes of the nonuniform transforms (rows of the x
// passes; entries y and lines z of the y passes; entries z of the z passes).
fsib::PassMasks mask_x(const Plan& p) {
  fsib::PassMasks m;
  if (p.ninst > 1 && p.dim == 3) return m;  // 3D multi-instance plans run their passes dense
  m.rows = {p.rowmask, (int)p.nf[1], (int)p.nf[2], (int)p.tb[1], (int)p.tb[2], (int)p.nt[1]};
  if (p.ninst > 1) {  // 2D: rows of instance i follow one another, p.dim fields each
    m.rows.rpi = (int64_t)p.dim * p.nf[1] * p.nf[2];
    m.rows.istride = (int)(p.nt[1] * p.nt[2]);
  }
  return m;
}
fsib::PassMasks mask_y(const Plan& p, bool forward) {
  fsib::PassMasks m;
  if (p.ninst > 1 && p.dim == 3) return m;
  if (p.dim == 3) {
    m.line = {p.zmask, (int)p.nf[2], (int)p.tb[2], 1, 0};
    const fsib::StrideMask e{p.rowmask, (int)p.nf[2], (int)p.tb[2], (int)p.nt[1], (int)p.tb[1]};
    (forward ? m.ld : m.st) = e;
  } else if (p.ninst > 1) {
    // outer index o = field of instance o / p.dim: the mask block of that instance
    const fsib::StrideMask e{p.rowmask, INT32_MAX, p.dim, (int)p.nt[1], (int)p.tb[1]};
    (forward ? m.ld : m.st) = e;
  } else {
    const fsib::StrideMask e{p.rowmask, 1, 1, 0, (int)p.tb[1]};
    (forward ? m.ld : m.st) = e;
  }
  return m;
}
fsib::PassMasks mask_z(const Plan& p, bool forward) {
  fsib::PassMasks m;
  if (p.ninst > 1) return m;
  const fsib::StrideMask e{p.zmask, 1, 1, 0, (int)p.tb[2]};
  (forward ? m.ld : m.st) = e;
  return m;
}

fsib_status check_points(const Plan& p, int64_t M, const void* X) {
  if (M < 0 || M > p.max_points) return fail(FSIB_ERR_ARG, "M must be in [0, max_points]");
  if (M > 0 && !X) return fail(FSIB_ERR_ARG, "X is NULL");
  return FSIB_OK;
}

// Calls that take one point set: not on multi-instance plans.
fsib_status single_instance(const Plan& p) {
  if (p.ninst > 1) return fail(FSIB_ERR_STATE, "this call takes one instance; the plan holds ninst > 1");
  return FSIB_OK;
}

// Multi-instance plans: the instances are set, M covers them all, curve forces have >= 3 points each.
fsib_status check_instances(const Plan& p, int64_t M, const fsib_force* f) {
  if (p.ninst <= 1) return FSIB_OK;
  if (p.inst_off_h.empty()) return fail(FSIB_ERR_STATE, "fsib_plan_set_instances has not been called");
  if (M != p.inst_off_h[p.ninst]) return fail(FSIB_ERR_ARG, "M must equal the last instance offset");
  if (f && f->kind == FSIB_FORCE_CURVE_TENSION)
    for (int i = 0; i < p.ninst; ++i)
      if (p.inst_off_h[i + 1] - p.inst_off_h[i] < 3) return fail(FSIB_ERR_ARG, "curve tension needs >= 3 points per instance");
  return FSIB_OK;
}

// ---- transform pipelines ----
fsib_status type1_complex(Plan& p, int64_t M, const double* X, const void* c, void* fhat, double scale, hipStream_t st) {
  FSIB_HIP(fsib::launch_sort_points(p, M, X, st));
  FSIB_HIP(fsib::launch_spread(p, M, c, 0, st));
  const int64_t T = p.ntrans;
  if (p.dim == 3) {
    FSIB_HIP(fsib::launch_fft_c2c(p, p.grid, p.B1, (int)p.nf[0], -1, 1, T * p.nf[2] * p.nf[1], (int)p.nf[0],
                                  (int)p.nf[0], (int)p.N[0], (int)ceil_half(p.N[0]), nullptr, p.fac[0], 1.0, st,
                                  mask_x(p)));
    FSIB_HIP(fsib::launch_fft_c2c(p, p.B1, p.B2, (int)p.nf[1], -1, p.N[0], T * p.nf[2], (int)p.nf[1], (int)p.nf[1],
                                  (int)p.N[1], (int)ceil_half(p.N[1]), nullptr, p.fac[1], 1.0, st, mask_y(p, true)));
    FSIB_HIP(fsib::launch_fft_c2c(p, p.B2, fhat, (int)p.nf[2], -1, p.N[1] * p.N[0], T, (int)p.nf[2], (int)p.nf[2],
                                  (int)p.N[2], (int)ceil_half(p.N[2]), nullptr, p.fac[2], scale, st, mask_z(p, true)));
  } else {
    FSIB_HIP(fsib::launch_fft_c2c(p, p.grid, p.B1, (int)p.nf[0], -1, 1, T * p.nf[1], (int)p.nf[0], (int)p.nf[0],
                                  (int)p.N[0], (int)ceil_half(p.N[0]), nullptr, p.fac[0], 1.0, st, mask_x(p)));
    FSIB_HIP(fsib::launch_fft_c2c(p, p.B1, fhat, (int)p.nf[1], -1, p.N[0], T, (int)p.nf[1], (int)p.nf[1], (int)p.N[1],
                                  (int)ceil_half(p.N[1]), nullptr, p.fac[1], scale, st, mask_y(p, true)));
  }
  return FSIB_OK;
}

fsib_status type2_complex(Plan& p, int64_t M, const double* X, const void* fhat, void* c, hipStream_t st) {
  FSIB_HIP(fsib::launch_sort_points(p, M, X, st));
  const int64_t T = p.ntrans;
  if (p.dim == 3) {
    FSIB_HIP(fsib::launch_fft_c2c(p, fhat, p.B2, (int)p.nf[2], +1, p.N[1] * p.N[0], T, (int)p.N[2],
                                  (int)ceil_half(p.N[2]), (int)p.nf[2], (int)p.nf[2], p.fac[2], nullptr, 1.0, st,
                                  mask_z(p, false)));
    FSIB_HIP(fsib::launch_fft_c2c(p, p.B2, p.B1, (int)p.nf[1], +1, p.N[0], T * p.nf[2], (int)p.N[1],
                                  (int)ceil_half(p.N[1]), (int)p.nf[1], (int)p.nf[1], p.fac[1], nullptr, 1.0, st,
                                  mask_y(p, false)));
    FSIB_HIP(fsib::launch_fft_c2c(p, p.B1, p.grid, (int)p.nf[0], +1, 1, T * p.nf[2] * p.nf[1], (int)p.N[0],
                                  (int)ceil_half(p.N[0]), (int)p.nf[0], (int)p.nf[0], p.fac[0], nullptr, 1.0, st,
                                  mask_x(p)));
  } else {
    FSIB_HIP(fsib::launch_fft_c2c(p, fhat, p.B1, (int)p.nf[1], +1, p.N[0], T, (int)p.N[1], (int)ceil_half(p.N[1]),
                                  (int)p.nf[1], (int)p.nf[1], p.fac[1], nullptr, 1.0, st, mask_y(p, false)));
    FSIB_HIP(fsib::launch_fft_c2c(p, p.B1, p.grid, (int)p.nf[0], +1, 1, T * p.nf[1], (int)p.N[0],
                                  (int)ceil_half(p.N[0]), (int)p.nf[0], (int)p.nf[0], p.fac[0], nullptr, 1.0, st,
                                  mask_x(p)));
  }
  FSIB_HIP(fsib::launch_interp(p, M, c, 0, st));
  return FSIB_OK;
}

// real vector strengths (sorted point set already in place) -> dim half spectra
fsib_status force_spread_sorted(Plan& p, int64_t M, const void* S_, void* fhat, double scale, hipStream_t st) {
  FSIB_HIP(fsib::launch_spread(p, M, S_, p.dim, st));
  const int64_t d = (int64_t)p.dim * p.ninst;  // real fields of all instances
  if (p.dim == 3) {
    FSIB_HIP(fsib::launch_fft_r2c_x(p, p.grid, p.B1, (int)p.nf[0], d * p.nf[2] * p.nf[1], (int)p.Hx, p.fac[0], 1.0, st,
                                    mask_x(p)));
    FSIB_HIP(fsib::launch_fft_c2c(p, p.B1, p.B2, (int)p.nf[1], -1, p.Hx, d * p.nf[2], (int)p.nf[1], (int)p.nf[1],
                                  (int)p.N[1], (int)ceil_half(p.N[1]), nullptr, p.fac[1], 1.0, st, mask_y(p, true)));
    FSIB_HIP(fsib::launch_fft_c2c(p, p.B2, fhat, (int)p.nf[2], -1, p.N[1] * p.Hx, d, (int)p.nf[2], (int)p.nf[2],
                                  (int)p.N[2], (int)ceil_half(p.N[2]), nullptr, p.fac[2], scale, st, mask_z(p, true)));
  } else {
    FSIB_HIP(fsib::launch_fft_r2c_x(p, p.grid, p.B1, (int)p.nf[0], d * p.nf[1], (int)p.Hx, p.fac[0], 1.0, st,
                                    mask_x(p)));
    FSIB_HIP(fsib::launch_fft_c2c(p, p.B1, fhat, (int)p.nf[1], -1, p.Hx, d, (int)p.nf[1], (int)p.nf[1], (int)p.N[1],
                                  (int)ceil_half(p.N[1]), nullptr, p.fac[1], scale, st, mask_y(p, true)));
  }
  return FSIB_OK;
}

// dim half spectra -> real vector velocity at the sorted point set
// U at the sorted points from uhat; move (nullable): X += move_a U in the same pass.
fsib_status velocity_interp_sorted(Plan& p, int64_t M, const void* uhat, void* U, hipStream_t st,
                                   double* move = nullptr, double move_a = 0) {
  const int64_t d = (int64_t)p.dim * p.ninst;  // real fields of all instances
  if (p.dim == 3) {
    FSIB_HIP(fsib::launch_fft_c2c(p, uhat, p.B2, (int)p.nf[2], +1, p.N[1] * p.Hx, d, (int)p.N[2],
                                  (int)ceil_half(p.N[2]), (int)p.nf[2], (int)p.nf[2], p.fac[2], nullptr, 1.0, st,
                                  mask_z(p, false)));
    FSIB_HIP(fsib::launch_fft_c2c(p, p.B2, p.B1, (int)p.nf[1], +1, p.Hx, d * p.nf[2], (int)p.N[1],
                                  (int)ceil_half(p.N[1]), (int)p.nf[1], (int)p.nf[1], p.fac[1], nullptr, 1.0, st,
                                  mask_y(p, false)));
    FSIB_HIP(fsib::launch_fft_c2r_x(p, p.B1, p.grid, (int)p.nf[0], d * p.nf[2] * p.nf[1], (int)p.Hx, p.fac[0], 1.0, st,
                                    mask_x(p)));
  } else {
    FSIB_HIP(fsib::launch_fft_c2c(p, uhat, p.B1, (int)p.nf[1], +1, p.Hx, d, (int)p.N[1], (int)ceil_half(p.N[1]),
                                  (int)p.nf[1], (int)p.nf[1], p.fac[1], nullptr, 1.0, st, mask_y(p, false)));
    FSIB_HIP(fsib::launch_fft_c2r_x(p, p.B1, p.grid, (int)p.nf[0], d * p.nf[1], (int)p.Hx, p.fac[0], 1.0, st,
                                    mask_x(p)));
  }
  FSIB_HIP(fsib::launch_interp(p, M, U, p.dim, st, move, move_a));
  return FSIB_OK;
}

// FFT stages of the fused products x pass on 192-point lines: the tuning knob, else two (the faster
// kernel alone: 95 against 119 us per launch at 128^3 in FP64) unless an FP64 first half step runs
// it beside its point side.  There the point side (sorting, spreading, the type-1 passes) is the
// step's critical path, and the two-stage kernel's higher draw on memory and LDS slows it more than
// the products gain: 128^3 FP64 steps measured 1.113 ms with three stages in the first half and two
// in the second, 1.123 with three in both, 1.141 with two in both, 1.152 with two then three.
static int products_stages(const Plan& p, bool beside_point_side) {
  if (p.nl_stages != 0) return p.nl_stages;
  return p.prec == FSIB_F64 && beside_point_side ? 3 : 2;
}

// dealiased products of the field uhat (dim half spectra) -> p.pihat (nprod half spectra):
// inverse passes along z and y onto the dealiasing grid, the fused x pass (inverse transform,
// products, forward transform), forward passes along y and z back to K_N.  With last = false the
// pass along z is left out (the products wait in p.D1 for the pass fused with the update).
// beside_point_side: the first half step's point side runs concurrently (picks the x-pass kernel).
fsib_status dealiased_products(Plan& p, const void* uhat, hipStream_t st, bool last = true,
                               bool beside_point_side = false) {
  const int stages = products_stages(p, beside_point_side);
  const int64_t d = p.dim, np = p.nprod();
  if (p.dim == 3) {
    FSIB_HIP(fsib::launch_fft_c2c(p, uhat, p.D1, (int)p.nd[2], +1, p.N[1] * p.Hx, d, (int)p.N[2],
                                  (int)ceil_half(p.N[2]), (int)p.nd[2], (int)p.nd[2], nullptr, nullptr, 1.0, st));
    FSIB_HIP(fsib::launch_fft_c2c(p, p.D1, p.D2, (int)p.nd[1], +1, p.Hx, d * p.nd[2], (int)p.N[1],
                                  (int)ceil_half(p.N[1]), (int)p.nd[1], (int)p.nd[1], nullptr, nullptr, 1.0, st));
    FSIB_HIP(fsib::launch_nl_xpass(p, p.D2, p.prod, stages, st));
    FSIB_HIP(fsib::launch_fft_c2c(p, p.prod, p.D1, (int)p.nd[1], -1, p.Hx, np * p.nd[2], (int)p.nd[1], (int)p.nd[1],
                                  (int)p.N[1], (int)ceil_half(p.N[1]), nullptr, nullptr, 1.0, st));
    if (last)
      FSIB_HIP(fsib::launch_fft_c2c(p, p.D1, p.pihat, (int)p.nd[2], -1, p.N[1] * p.Hx, np, (int)p.nd[2],
                                    (int)p.nd[2], (int)p.N[2], (int)ceil_half(p.N[2]), nullptr, nullptr, 1.0, st));
  } else {
    FSIB_HIP(fsib::launch_fft_c2c(p, uhat, p.D2, (int)p.nd[1], +1, p.Hx, d, (int)p.N[1], (int)ceil_half(p.N[1]),
                                  (int)p.nd[1], (int)p.nd[1], nullptr, nullptr, 1.0, st));
    FSIB_HIP(fsib::launch_nl_xpass(p, p.D2, p.prod, stages, st));
    FSIB_HIP(fsib::launch_fft_c2c(p, p.prod, p.pihat, (int)p.nd[1], -1, p.Hx, np, (int)p.nd[1], (int)p.nd[1],
                                  (int)p.N[1], (int)ceil_half(p.N[1]), nullptr, nullptr, 1.0, st));
  }
  return FSIB_OK;
}

// Navier-Stokes update (mode FLUID_NS_HALF or FLUID_NS_FULL) uout <- update(fhat, uin) with the dealiased
// products of `field`; `ev` (when not null) is waited for before anything reads fhat.  Plans with 128
// modes and 192 dealiasing points along z run the products' last pass and the update as one kernel.
// beside_point_side as for dealiased_products.
fsib_status ns_update(Plan& p, int mode, const fsib_fluid_params& prm, const void* field, const void* fhat,
                      const void* uin, void* uout, hipEvent_t ev, hipStream_t st, bool beside_point_side = false) {
  const bool fused = fsib::products_z_fluid_fits(p);
  FSIB_TRY(dealiased_products(p, field, st, !fused, beside_point_side));
  if (ev) FSIB_HIP(hipStreamWaitEvent(st, ev, 0));
  if (fused)
    FSIB_HIP(fsib::launch_products_z_fluid(p, mode, prm, fhat, uin, uout, st));
  else
    FSIB_HIP(fsib::launch_fluid_update(p, mode, prm, fhat, uin, uout, st));
  return FSIB_OK;
}

fsib_status fluid_impl(Plan& p, const fsib_fluid_params& prm, const void* fhat, void* uhat, void* umid, hipStream_t st) {
  if (prm.model == FSIB_STOKES) {
    FSIB_HIP(fsib::launch_fluid_update(p, fsib::FLUID_STOKES, prm, fhat, nullptr, uhat, st));
    if (umid)
      FSIB_HIP(hipMemcpyAsync(umid, uhat, (size_t)p.dim * p.ninst * p.modes_half() * 2 * p.real_size(),
                              hipMemcpyDeviceToDevice, st));
    return FSIB_OK;
  }
  void* mid = umid ? umid : p.uhat_mid;
  FSIB_TRY(ns_update(p, fsib::FLUID_NS_HALF, prm, uhat, fhat, uhat, mid, nullptr, st));
  FSIB_TRY(ns_update(p, fsib::FLUID_NS_FULL, prm, mid, fhat, uhat, uhat, nullptr, st));
  return FSIB_OK;
}

fsib_status check_fluid(const Plan& p, const fsib_fluid_params* prm) {
  if (!p.fluid) return fail(FSIB_ERR_STATE, "plan was created without fluid = 1");
  if (!prm) return fail(FSIB_ERR_ARG, "params is NULL");
  if (prm->model != FSIB_STOKES && prm->model != FSIB_NAVIER_STOKES) return fail(FSIB_ERR_ARG, "unknown model");
  if (!(prm->mu > 0) || !std::isfinite(prm->mu)) return fail(FSIB_ERR_ARG, "mu must be positive");
  if (prm->model == FSIB_NAVIER_STOKES) {
    if (!p.ns) return fail(FSIB_ERR_STATE, "plan was created without navier_stokes = 1");
    if (!(prm->rho > 0) || !std::isfinite(prm->rho)) return fail(FSIB_ERR_ARG, "rho must be positive");
  }
  if (!std::isfinite(prm->dt)) return fail(FSIB_ERR_ARG, "dt must be finite");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(prm->body[a])) return fail(FSIB_ERR_ARG, "body force must be finite");
  return FSIB_OK;
}

fsib_status check_force(const fsib_force* f, int dim, int64_t M) {
  if (!f) return fail(FSIB_ERR_ARG, "force is NULL");
  if (!std::isfinite(f->K)) return fail(FSIB_ERR_ARG, "force K must be finite");
  if (f->kind == FSIB_FORCE_CURVE_TENSION) {
    if (dim != 2) return fail(FSIB_ERR_ARG, "curve tension needs dim = 2");
    if (M > 0 && M < 3) return fail(FSIB_ERR_ARG, "curve tension needs M >= 3");
    return FSIB_OK;
  }
  if (f->kind == FSIB_FORCE_SURFACE_TENSION) {
    if (dim != 3) return fail(FSIB_ERR_ARG, "surface tension needs dim = 3");
    if (M > 0 && (!f->tris || !f->v2t_ptr || !f->v2t_idx || f->ntris <= 0))
      return fail(FSIB_ERR_ARG, "surface tension needs tris and the vertex-triangle CSR");
    return FSIB_OK;
  }
  if (f->kind == FSIB_FORCE_EDGE_SPRINGS) {
    if (M > 0 && (!f->v2t_ptr || !f->v2t_idx || !f->aux))
      return fail(FSIB_ERR_ARG, "edge springs need the neighbour CSR and the stiffness per entry (aux)");
    return FSIB_OK;
  }
  if (f->kind == FSIB_FORCE_TARGET) {
    if (M > 0 && !f->aux) return fail(FSIB_ERR_ARG, "target points need the targets (aux)");
    return FSIB_OK;
  }
  return fail(FSIB_ERR_ARG, "unknown force kind");
}

// Stokes boundary velocity at X: force, spread, Stokeslet, interp.  uhat receives the field.
fsib_status stokes_velocity(Plan& p, const fsib_fluid_params& prm, const fsib_force& f, int64_t M, const double* X,
                            void* U, void* uhat, hipStream_t st) {
  const double Ld = p.dim == 3 ? p.L * p.L * p.L : p.L * p.L;
  FSIB_HIP(fsib::launch_force_strengths(p, f, M, X, p.F64, p.S, st));
  FSIB_HIP(fsib::launch_sort_points(p, M, X, st, p.S));
  FSIB_TRY(force_spread_sorted(p, M, p.S, p.fhat, 1.0 / Ld, st));
  FSIB_HIP(fsib::launch_fluid_update(p, fsib::FLUID_STOKES, prm, p.fhat, nullptr, uhat, st));
  FSIB_TRY(velocity_interp_sorted(p, M, uhat, U, st));
  return FSIB_OK;
}

// ---- groups: Stokes steps of several plans, every stage one launch over all of them ----
// The transforms of force_spread_sorted (fine grids -> p.fhat, scaled by 1/L^d) and of
// velocity_interp_sorted (uhat[g] -> fine grids) for the plans of a group.
fsib_status group_spread_ffts(const std::vector<Plan*>& ps, hipStream_t st) {
  std::vector<fsib::FftCall> x, y, z;
  for (Plan* q : ps) {
    Plan& p = *q;
    const int64_t d = (int64_t)p.dim * p.ninst;
    const double scale = 1.0 / (p.dim == 3 ? p.L * p.L * p.L : p.L * p.L);
    const int nf0 = (int)p.nf[0], nf1 = (int)p.nf[1], nf2 = (int)p.nf[2], hx = (int)p.Hx;
    if (p.dim == 3) {
      x.push_back({&p, p.grid, p.B1, nf0, -1, 1, d * p.nf[2] * p.nf[1], nf0, nf0, hx, hx, nullptr, p.fac[0], 1.0,
                   mask_x(p)});
      y.push_back({&p, p.B1, p.B2, nf1, -1, p.Hx, d * p.nf[2], nf1, nf1, (int)p.N[1], (int)ceil_half(p.N[1]), nullptr,
                   p.fac[1], 1.0, mask_y(p, true)});
      z.push_back({&p, p.B2, p.fhat, nf2, -1, p.N[1] * p.Hx, d, nf2, nf2, (int)p.N[2], (int)ceil_half(p.N[2]), nullptr,
                   p.fac[2], scale, mask_z(p, true)});
    } else {
      x.push_back({&p, p.grid, p.B1, nf0, -1, 1, d * p.nf[1], nf0, nf0, hx, hx, nullptr, p.fac[0], 1.0, mask_x(p)});
      y.push_back({&p, p.B1, p.fhat, nf1, -1, p.Hx, d, nf1, nf1, (int)p.N[1], (int)ceil_half(p.N[1]), nullptr, p.fac[1],
                   scale, mask_y(p, true)});
    }
  }
  FSIB_HIP(fsib::launch_fft_x_group(x, true, st));
  FSIB_HIP(fsib::launch_fft_c2c_group(y, st));
  FSIB_HIP(fsib::launch_fft_c2c_group(z, st));
  return FSIB_OK;
}

fsib_status group_interp_ffts(const std::vector<Plan*>& ps, void* const* uhat, hipStream_t st) {
  std::vector<fsib::FftCall> x, y, z;
  for (size_t g = 0; g < ps.size(); ++g) {
    Plan& p = *ps[g];
    const int64_t d = (int64_t)p.dim * p.ninst;
    const int nf0 = (int)p.nf[0], nf1 = (int)p.nf[1], nf2 = (int)p.nf[2], hx = (int)p.Hx;
    if (p.dim == 3) {
      z.push_back({&p, uhat[g], p.B2, nf2, +1, p.N[1] * p.Hx, d, (int)p.N[2], (int)ceil_half(p.N[2]), nf2, nf2,
                   p.fac[2], nullptr, 1.0, mask_z(p, false)});
      y.push_back({&p, p.B2, p.B1, nf1, +1, p.Hx, d * p.nf[2], (int)p.N[1], (int)ceil_half(p.N[1]), nf1, nf1, p.fac[1],
                   nullptr, 1.0, mask_y(p, false)});
      x.push_back({&p, p.B1, p.grid, nf0, +1, 1, d * p.nf[2] * p.nf[1], hx, hx, nf0, nf0, p.fac[0], nullptr, 1.0,
                   mask_x(p)});
    } else {
      y.push_back({&p, uhat[g], p.B1, nf1, +1, p.Hx, d, (int)p.N[1], (int)ceil_half(p.N[1]), nf1, nf1, p.fac[1],
                   nullptr, 1.0, mask_y(p, false)});
      x.push_back({&p, p.B1, p.grid, nf0, +1, 1, d * p.nf[1], hx, hx, nf0, nf0, p.fac[0], nullptr, 1.0, mask_x(p)});
    }
  }
  FSIB_HIP(fsib::launch_fft_c2c_group(z, st));
  FSIB_HIP(fsib::launch_fft_c2c_group(y, st));
  FSIB_HIP(fsib::launch_fft_x_group(x, false, st));
  return FSIB_OK;
}

// stokes_velocity for every plan of a group: U[g] at X[g], uhat[g] the field; mv (nullable): position
// updates from U done by the interpolation pass.
fsib_status group_stokes_velocity(const std::vector<Plan*>& ps, const fsib_fluid_params* prm, const fsib_force* f,
                                  const int64_t* M, const double* const* X, void* const* U, void* const* uhat,
                                  hipStream_t st, const fsib::GroupMove* mv = nullptr) {
  const size_t n = ps.size();
  std::vector<const void*> S(n);
  for (size_t g = 0; g < n; ++g) S[g] = ps[g]->S;
  FSIB_HIP(fsib::launch_force_strengths_group(ps, f, M, X, st));
  FSIB_HIP(fsib::launch_sort_points_group(ps, M, X, st, S.data()));
  FSIB_HIP(fsib::launch_spread_group(ps, M, S.data(), st));
  FSIB_TRY(group_spread_ffts(ps, st));
  FSIB_HIP(fsib::launch_fluid_stokes_group(ps, prm, uhat, st));
  FSIB_TRY(group_interp_ffts(ps, uhat, st));
  FSIB_HIP(fsib::launch_interp_group(ps, M, U, st, mv));
  return FSIB_OK;
}

}  // namespace

struct fsib_group_s {
  std::vector<fsib_plan> plans;
  std::vector<Plan*> ps;
};

namespace fsib {

fsib_status report(fsib_status s, const char* msg) { return fail(s, msg); }

// Per-call buffers of a type-1 transform carved from one device block (each 256-byte aligned), in the
// sizes build_plan gives them but for M points instead of max_points.  With base == nullptr only the
// size is computed.  The plan's tables (kernel pieces, deconvolution factors, twiddles, flag) stay.
struct TransformBuffers {
  int* counts; int* offsets; int* pt_bin; int* pt_rank; int* det_key; int* s_idx; uint32_t* s_i0; void* s_y;
  void* s_str; int* scan_part; uint8_t* rowmask; uint8_t* zmask; int* tile_parts; int* part_off; int* work;
  int* tile_slot; int* slot_ctr; int* split_list; void* split_scratch; void* grid; void* B1; void* B2;
  int64_t work_blocks, split_slots;
};

static int64_t carve_transform_buffers(const Plan& p, int64_t M, char* base, TransformBuffers& b) {
  int64_t off = 0;
  auto take = [&](auto*& ptr, int64_t bytes) {
    if (bytes <= 0) bytes = 256;
    ptr = base ? reinterpret_cast<std::remove_reference_t<decltype(ptr)>>(base + off) : nullptr;
    off += (bytes + 255) / 256 * 256;
  };
  const int64_t rs = (int64_t)p.real_size(), cs = 2 * rs, d = p.dim;
  const int64_t Mx = M > 0 ? M : 1;
  take(b.counts, (p.nbt + 1) * 4);
  take(b.offsets, (p.nbt + 1) * 4);
  take(b.pt_bin, Mx * 4);
  take(b.pt_rank, Mx * 4);
  b.det_key = nullptr;
  if (p.deterministic) take(b.det_key, Mx * 4);
  take(b.s_idx, Mx * 4);
  take(b.s_i0, Mx * 4);
  take(b.s_y, Mx * d * rs);
  take(b.s_str, Mx * (2 * p.ntrans > d ? 2 * p.ntrans : d) * rs);
  take(b.scan_part, scan_segments(p.nbt) * 4);
  take(b.rowmask, p.nt[1] * p.nt[2]);
  take(b.zmask, p.nt[2]);
  int64_t reach = 1;
  for (int a = 0; a < p.dim; ++a) reach *= p.qn[a] + 1;
  const int64_t visits = Mx * reach;
  b.work_blocks = p.nbt + visits / p.split + 1;
  b.split_slots = 2 * visits / p.split + 2;
  const int64_t nch_bytes = 2 * rs > d * rs ? 2 * rs : d * rs;
  take(b.tile_parts, p.nbt * 4);
  take(b.part_off, (p.nbt + 1) * 4);
  take(b.work, b.work_blocks * 8);
  take(b.tile_slot, p.nbt * 4);
  take(b.slot_ctr, 256);
  take(b.split_list, (b.split_slots / 2 + 1) * 4);
  take(b.split_scratch, (int64_t)p.ntrans * b.split_slots * 1024 * nch_bytes);
  take(b.grid, (int64_t)p.ntrans * p.fine_cells() * cs);
  take(b.B1, p.dim == 3 ? (int64_t)p.ntrans * p.nf[2] * p.nf[1] * p.N[0] * cs : (int64_t)p.ntrans * p.nf[1] * p.N[0] * cs);
  take(b.B2, p.dim == 3 ? (int64_t)p.ntrans * p.nf[2] * p.N[1] * p.N[0] * cs : 0);
  return off;
}

// The plan's per-call buffer fields exchanged with b (twice restores them).
static void swap_transform_buffers(Plan& p, TransformBuffers& b) {
  std::swap(p.counts, b.counts);
  std::swap(p.offsets, b.offsets);
  std::swap(p.pt_bin, b.pt_bin);
  std::swap(p.pt_rank, b.pt_rank);
  std::swap(p.det_key, b.det_key);
  std::swap(p.s_idx, b.s_idx);
  std::swap(p.s_i0, b.s_i0);
  std::swap(p.s_y, b.s_y);
  std::swap(p.s_str, b.s_str);
  std::swap(p.scan_part, b.scan_part);
  std::swap(p.rowmask, b.rowmask);
  std::swap(p.zmask, b.zmask);
  std::swap(p.tile_parts, b.tile_parts);
  std::swap(p.part_off, b.part_off);
  std::swap(p.work, b.work);
  std::swap(p.tile_slot, b.tile_slot);
  std::swap(p.slot_ctr, b.slot_ctr);
  std::swap(p.split_list, b.split_list);
  std::swap(p.split_scratch, b.split_scratch);
  std::swap(p.grid, b.grid);
  std::swap(p.B1, b.B1);
  std::swap(p.B2, b.B2);
  std::swap(p.work_blocks, b.work_blocks);
  std::swap(p.split_slots, b.split_slots);
}

fsib_status spread_in_workspace(fsib_plan plan, int device, int64_t M, const double* X, const void* c, void* fhat,
                                double scale, void* stream, void* ws, int64_t ws_bytes) {
  if (!plan) return fail(FSIB_ERR_ARG, "plan is NULL");
  Plan& p = plan->p;
  if (device != p.device) return fail(FSIB_ERR_ARG, "the current device is not the plan's device");
  if (p.fluid) return fail(FSIB_ERR_STATE, "this call takes a plan created with fluid = 0");
  if (M < 0 || M > ((int64_t)1 << 30)) return fail(FSIB_ERR_ARG, "M must be in [0, 2^30]");
  if (M > 0 && (!X || !c)) return fail(FSIB_ERR_ARG, "X and c must not be NULL");
  if (!fhat) return fail(FSIB_ERR_ARG, "fhat is NULL");
  if (!std::isfinite(scale)) return fail(FSIB_ERR_ARG, "scale must be finite");
  TransformBuffers b;
  const int64_t need = carve_transform_buffers(p, M, nullptr, b);
  if (need > ws_bytes)
    return fail(FSIB_ERR_ARG, "this transform needs " + std::to_string(need) + " bytes of scratch; the static " +
                                  "scratch holds " + std::to_string(ws_bytes) + " bytes (fewer points, modes or ntrans)");
  carve_transform_buffers(p, M, static_cast<char*>(ws), b);
  swap_transform_buffers(p, b);
  const bool counts_zero = p.counts_zero;
  const int parts_split = p.parts_split;
  p.counts_zero = false;  // the workspace's counts hold whatever the last call left
  const fsib_status s = type1_complex(p, M, X, c, fhat, scale, S(stream));
  swap_transform_buffers(p, b);
  p.counts_zero = counts_zero;  // the plan's own counts and tiles' parts are untouched
  p.parts_split = parts_split;
  return s;
}

}  // namespace fsib

extern "C" {

const char* fsib_version(void) { return "fsib-mi355x 0.1.0 (gfx950)"; }

const char* fsib_status_string(fsib_status s) {
  switch (s) {
    case FSIB_OK: return "ok";
    case FSIB_ERR_ARG: return "invalid argument";
    case FSIB_ERR_TOL: return "tolerance not reachable in this precision";
    case FSIB_ERR_NO_DEVICE: return "no HIP device";
    case FSIB_ERR_OOM: return "out of device memory";
    case FSIB_ERR_HIP: return "HIP runtime error";
    case FSIB_ERR_NONFINITE: return "non-finite position seen";
    case FSIB_ERR_STATE: return "plan lacks the workspace for this call";
  }
  return "unknown status";
}

const char* fsib_last_error(void) { return g_last_error.c_str(); }

int fsib_device_count(void) {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess) return 0;
  return n;
}

fsib_status fsib_plan_create(const fsib_plan_opts* opts, fsib_plan* out) {
  if (!out) return fail(FSIB_ERR_ARG, "out is NULL");
  FSIB_TRY(validate_opts(opts));
  if (fsib_device_count() <= 0) return fail(FSIB_ERR_NO_DEVICE, "no HIP device visible");
  fsib_plan h = new (std::nothrow) fsib_plan_s();
  if (!h) return fail(FSIB_ERR_OOM, "host allocation failed");
  fsib_status s = build_plan(h->p, opts);
  if (s != FSIB_OK) {
    free_plan(h->p);
    delete h;
    return s;
  }
  *out = h;
  return FSIB_OK;
}

fsib_status fsib_plan_set_instances(fsib_plan plan, const int64_t* offsets) {
  if (!plan) return fail(FSIB_ERR_ARG, "plan is NULL");
  Plan& p = plan->p;
  if (p.ninst <= 1) return fail(FSIB_ERR_STATE, "the plan holds one instance");
  if (!offsets) return fail(FSIB_ERR_ARG, "offsets is NULL");
  if (offsets[0] != 0) return fail(FSIB_ERR_ARG, "offsets[0] must be 0");
  for (int i = 0; i < p.ninst; ++i)
    if (offsets[i + 1] < offsets[i]) return fail(FSIB_ERR_ARG, "offsets must be non-decreasing");
  if (offsets[p.ninst] > p.max_points) return fail(FSIB_ERR_ARG, "offsets[ninst] exceeds max_points");
  FSIB_HIP(hipMemcpy(p.inst_off, offsets, (size_t)(p.ninst + 1) * sizeof(int64_t), hipMemcpyHostToDevice));
  p.inst_off_h.assign(offsets, offsets + p.ninst + 1);
  return FSIB_OK;
}

fsib_status fsib_plan_destroy(fsib_plan plan) {
  if (!plan) return fail(FSIB_ERR_ARG, "plan is NULL");
  (void)hipDeviceSynchronize();
  free_plan(plan->p);
  delete plan;
  return FSIB_OK;
}

fsib_status fsib_plan_info(fsib_plan plan, fsib_plan_info_t* info) {
  if (!plan || !info) return fail(FSIB_ERR_ARG, "plan or info is NULL");
  const Plan& p = plan->p;
  info->w = p.w;
  info->beta = p.beta;
  info->degree = p.deg;
  for (int a = 0; a < 3; ++a) {
    info->n_fine[a] = p.nf[a];
    info->n_dealias[a] = p.ns ? p.nd[a] : 0;
    info->tile[a] = p.tb[a];
  }
  info->workspace_bytes = p.ws_bytes;
  return FSIB_OK;
}

fsib_status fsib_plan_check(fsib_plan plan, void* stream) {
  if (!plan) return fail(FSIB_ERR_ARG, "plan is NULL");
  int flag = 0;
  FSIB_HIP(hipMemcpyAsync(&flag, plan->p.flag, sizeof(int), hipMemcpyDeviceToHost, S(stream)));
  FSIB_HIP(hipStreamSynchronize(S(stream)));
  if (flag) {
    FSIB_HIP(hipMemsetAsync(plan->p.flag, 0, sizeof(int), S(stream)));
    FSIB_HIP(hipStreamSynchronize(S(stream)));
    return fail(FSIB_ERR_NONFINITE, "a non-finite position was seen (treated as x = 0)");
  }
  return FSIB_OK;
}

fsib_status fsib_plan_tuning(fsib_plan plan, fsib_tuning* t, int get) {
  if (!plan) return fail(FSIB_ERR_ARG, "plan is NULL");
  if (!t) return fail(FSIB_ERR_ARG, "tuning is NULL");
  Plan& p = plan->p;
  if (get) {
    t->xcd_chunk_interp = p.xcd_chunk_interp;
    t->xcd_chunk_spread = p.xcd_chunk_spread;
    t->split = p.split;
    t->overlap = p.overlap;
    t->interp_points = p.interp_points;
    t->spread_threads = p.spread_threads;
    t->nl_stages = p.nl_stages;
    return FSIB_OK;
  }
  if (t->xcd_chunk_interp < 0 || t->xcd_chunk_interp > 4096 || t->xcd_chunk_spread < 0 || t->xcd_chunk_spread > 4096)
    return fail(FSIB_ERR_ARG, "XCD chunks must be in [0, 4096]");
  if (t->split < p.split_alloc || t->split > (1 << 20))
    return fail(FSIB_ERR_ARG, "split must be in [the creation value, 1 << 20]");
  if (t->overlap != 0 && t->overlap != 1) return fail(FSIB_ERR_ARG, "overlap must be 0 or 1");
  if (t->interp_points != 1 && t->interp_points != 2 && t->interp_points != 4 && t->interp_points != 8 &&
      t->interp_points != 16)
    return fail(FSIB_ERR_ARG, "interp_points must be 1, 2, 4, 8 or 16");
  const int sthr = t->spread_threads;
  if (p.dim == 2 ? (sthr != 0 && sthr != 64 && sthr != 128 && sthr != 256) : (sthr != 0 && sthr != 256))
    return fail(FSIB_ERR_ARG, "spread_threads must be 0, 64, 128 or 256 (2D) or 0 or 256 (3D)");
  if (t->nl_stages != 0 && t->nl_stages != 2 && t->nl_stages != 3)
    return fail(FSIB_ERR_ARG, "nl_stages must be 0, 2 or 3");
  p.nl_stages = t->nl_stages;
  p.spread_threads = sthr;
  p.interp_points = t->interp_points;
  p.overlap = t->overlap;
  p.xcd_chunk_interp = t->xcd_chunk_interp;
  p.xcd_chunk_spread = t->xcd_chunk_spread;
  p.split = t->split;
  return FSIB_OK;
}

fsib_status fsib_plan_profile(fsib_plan plan, int kernel_class, int max_launches) {
  if (!plan) return fail(FSIB_ERR_ARG, "plan is NULL");
  Plan& p = plan->p;
  if (kernel_class != -1 && (kernel_class < FSIB_PROF_FFT_STRIDED || kernel_class > FSIB_PROF_NL_X))
    return fail(FSIB_ERR_ARG, "unknown kernel class");
  if (max_launches < 0 || max_launches > (1 << 20)) return fail(FSIB_ERR_ARG, "max_launches out of range");
  FSIB_HIP(hipDeviceSynchronize());
  for (hipEvent_t e : p.prof_ev) (void)hipEventDestroy(e);
  p.prof_ev.clear();
  p.prof_used = 0;
  p.prof_bytes = 0.0;
  p.prof_class = -1;
  if (kernel_class == -1 || max_launches == 0) return FSIB_OK;
  p.prof_ev.resize(2 * (size_t)max_launches);
  for (auto& e : p.prof_ev) FSIB_HIP(hipEventCreate(&e));
  p.prof_class = kernel_class;
  return FSIB_OK;
}

fsib_status fsib_plan_profile_read(fsib_plan plan, double* total_ms, int64_t* launches, double* bytes) {
  if (!plan || !total_ms || !launches || !bytes) return fail(FSIB_ERR_ARG, "NULL argument");
  Plan& p = plan->p;
  double tot = 0.0;
  for (int i = 0; i < p.prof_used; ++i) {
    FSIB_HIP(hipEventSynchronize(p.prof_ev[2 * (size_t)i + 1]));
    float ms = 0.f;
    FSIB_HIP(hipEventElapsedTime(&ms, p.prof_ev[2 * (size_t)i], p.prof_ev[2 * (size_t)i + 1]));
    tot += ms;
  }
  *total_ms = tot;
  *launches = p.prof_used;
  *bytes = p.prof_bytes;
  p.prof_used = 0;
  p.prof_bytes = 0.0;
  return FSIB_OK;
}

fsib_status fsib_spread(fsib_plan plan, int64_t M, const double* X, const void* c, void* fhat, double scale,
                        void* stream) {
  if (!plan) return fail(FSIB_ERR_ARG, "plan is NULL");
  Plan& p = plan->p;
  FSIB_TRY(single_instance(p));
  FSIB_TRY(check_points(p, M, X));
  if (M > 0 && !c) return fail(FSIB_ERR_ARG, "c is NULL");
  if (!fhat) return fail(FSIB_ERR_ARG, "fhat is NULL");
  if (!std::isfinite(scale)) return fail(FSIB_ERR_ARG, "scale must be finite");
  return type1_complex(p, M, X, c, fhat, scale, S(stream));
}


fsib_status fsib_interp(fsib_plan plan, int64_t M, const double* X, const void* fhat, void* c, void* stream) {
  if (!plan) return fail(FSIB_ERR_ARG, "plan is NULL");
  Plan& p = plan->p;
  FSIB_TRY(single_instance(p));
  FSIB_TRY(check_points(p, M, X));
  if (!fhat) return fail(FSIB_ERR_ARG, "fhat is NULL");
  if (M > 0 && !c) return fail(FSIB_ERR_ARG, "c is NULL");
  return type2_complex(p, M, X, fhat, c, S(stream));
}

fsib_status fsib_spectral_scale(fsib_plan plan, int layout, int axis, double scale, const void* in, void* out,
                                void* stream) {
  if (!plan) return fail(FSIB_ERR_ARG, "plan is NULL");
  Plan& p = plan->p;
  FSIB_TRY(single_instance(p));
  if (layout != 0 && layout != 1) return fail(FSIB_ERR_ARG, "layout must be 0 (full spectra) or 1 (half spectra)");
  if (layout == 1 && !p.fluid) return fail(FSIB_ERR_STATE, "half spectra need a plan created with fluid = 1");
  if (axis < -1 || axis >= p.dim) return fail(FSIB_ERR_ARG, "axis must be -1 or in [0, dim)");
  if (!in || !out) return fail(FSIB_ERR_ARG, "in / out is NULL");
  if (!std::isfinite(scale)) return fail(FSIB_ERR_ARG, "scale must be finite");
  FSIB_HIP(fsib::launch_spectral_scale(p, layout, axis, scale, in, out, S(stream)));
  return FSIB_OK;
}

fsib_status fsib_grad_combine(fsib_plan plan, int64_t M, int kind, const void* u, const void* v, const void* u2,
                              const void* v2, double scale, double* gX, int axis, void* stream) {
  if (!plan) return fail(FSIB_ERR_ARG, "plan is NULL");
  Plan& p = plan->p;
  if (M < 0 || M > p.max_points) return fail(FSIB_ERR_ARG, "M out of range [0, max_points]");
  if (kind != 0 && kind != 1) return fail(FSIB_ERR_ARG, "kind must be 0 (complex) or 1 (real)");
  if (axis < 0 || axis >= p.dim) return fail(FSIB_ERR_ARG, "axis must be in [0, dim)");
  if (M > 0 && (!u || !v || !gX)) return fail(FSIB_ERR_ARG, "u / v / gX is NULL");
  if (M > 0 && kind == 1 && (!u2) != (!v2)) return fail(FSIB_ERR_ARG, "u2 and v2 must both be given or both NULL");
  if (!std::isfinite(scale)) return fail(FSIB_ERR_ARG, "scale must be finite");
  FSIB_HIP(fsib::launch_grad_combine(p, M, kind, u, v, kind == 1 ? u2 : nullptr, kind == 1 ? v2 : nullptr, scale, gX,
                                     axis, S(stream)));
  return FSIB_OK;
}

fsib_status fsib_force_spread(fsib_plan plan, int64_t M, const double* X, const void* S_, void* fhat_half, double scale,
                              void* stream) {
  if (!plan) return fail(FSIB_ERR_ARG, "plan is NULL");
  Plan& p = plan->p;
  if (!p.fluid) return fail(FSIB_ERR_STATE, "plan was created without fluid = 1");
  FSIB_TRY(check_points(p, M, X));
  FSIB_TRY(check_instances(p, M, nullptr));
  if (M > 0 && !S_) return fail(FSIB_ERR_ARG, "S is NULL");
  if (!fhat_half) return fail(FSIB_ERR_ARG, "fhat_half is NULL");
  if (!std::isfinite(scale)) return fail(FSIB_ERR_ARG, "scale must be finite");
  FSIB_HIP(fsib::launch_sort_points(p, M, X, S(stream), S_));
  return force_spread_sorted(p, M, S_, fhat_half, scale, S(stream));
}

fsib_status fsib_velocity_interp(fsib_plan plan, int64_t M, const double* X, const void* uhat_half, void* U,
                                 void* stream) {
  if (!plan) return fail(FSIB_ERR_ARG, "plan is NULL");
  Plan& p = plan->p;
  if (!p.fluid) return fail(FSIB_ERR_STATE, "plan was created without fluid = 1");
  FSIB_TRY(check_points(p, M, X));
  FSIB_TRY(check_instances(p, M, nullptr));
  if (!uhat_half) return fail(FSIB_ERR_ARG, "uhat_half is NULL");
  if (M > 0 && !U) return fail(FSIB_ERR_ARG, "U is NULL");
  FSIB_HIP(fsib::launch_sort_points(p, M, X, S(stream)));
  return velocity_interp_sorted(p, M, uhat_half, U, S(stream));
}

fsib_status fsib_fluid_step(fsib_plan plan, const fsib_fluid_params* params, const void* fhat_half, void* uhat_half,
                            void* uhat_mid, void* stream) {
  if (!plan) return fail(FSIB_ERR_ARG, "plan is NULL");
  Plan& p = plan->p;
  FSIB_TRY(check_fluid(p, params));
  if (!fhat_half || !uhat_half) return fail(FSIB_ERR_ARG, "fhat_half and uhat_half must not be NULL");
  return fluid_impl(p, *params, fhat_half, uhat_half, uhat_mid, S(stream));
}

fsib_status fsib_compute_force(const fsib_force* force, int dim, int64_t M, const double* X, double* F, void* stream) {
  if (dim != 2 && dim != 3) return fail(FSIB_ERR_ARG, "dim must be 2 or 3");
  if (M < 0) return fail(FSIB_ERR_ARG, "M must be >= 0");
  FSIB_TRY(check_force(force, dim, M));
  if (M > 0 && (!X || !F)) return fail(FSIB_ERR_ARG, "X and F must not be NULL");
  FSIB_HIP(fsib::launch_force(*force, dim, M, X, F, S(stream)));
  return FSIB_OK;
}

fsib_status fsib_force_jvp(const fsib_force* force, int dim, int64_t M, const double* X, const double* V, double* out,
                          void* stream) {
  if (dim != 2 && dim != 3) return fail(FSIB_ERR_ARG, "dim must be 2 or 3");
  if (M < 0) return fail(FSIB_ERR_ARG, "M must be >= 0");
  FSIB_TRY(check_force(force, dim, M));
  if (M > 0 && (!X || !V || !out)) return fail(FSIB_ERR_ARG, "X, V and out must not be NULL");
  if (M > 0 && (out == X || out == V)) return fail(FSIB_ERR_ARG, "out must not alias X or V");
  FSIB_HIP(fsib::launch_force_jvp(*force, dim, M, X, V, out, S(stream)));
  return FSIB_OK;
}

fsib_status fsib_spring_stiffness(int64_t M, const double* X0, const int32_t* tris, const int32_t* v2t_ptr,
                                  const int32_t* v2t_idx, const int32_t* nbr_ptr, const int32_t* nbr_idx,
                                  double* kij) {
  if (M < 0) return fail(FSIB_ERR_ARG, "M must be >= 0");
  if (M == 0) return FSIB_OK;
  if (!X0 || !tris || !v2t_ptr || !v2t_idx || !nbr_ptr || !nbr_idx || !kij)
    return fail(FSIB_ERR_ARG, "arrays must not be NULL");
  int* missing = nullptr;
  FSIB_HIP(hipMalloc(&missing, sizeof(int)));
  hipError_t e = hipMemset(missing, 0, sizeof(int));
  if (e == hipSuccess) e = fsib::launch_spring_stiffness(M, X0, tris, v2t_ptr, v2t_idx, nbr_ptr, nbr_idx, kij, missing,
                                                         nullptr);
  int h = 0;
  if (e == hipSuccess) e = hipMemcpy(&h, missing, sizeof(int), hipMemcpyDeviceToHost);
  (void)hipFree(missing);
  FSIB_HIP(e);
  if (h) return fail(FSIB_ERR_ARG, "a triangle edge is missing from the neighbour lists");
  return FSIB_OK;
}

fsib_status fsib_pressure(fsib_plan plan, const fsib_fluid_params* params, const void* fhat_half,
                          const void* uhat_half, void* phat_half, void* stream) {
  if (!plan) return fail(FSIB_ERR_ARG, "plan is NULL");
  Plan& p = plan->p;
  FSIB_TRY(single_instance(p));
  FSIB_TRY(check_fluid(p, params));
  if (!fhat_half || !phat_half) return fail(FSIB_ERR_ARG, "fhat_half and phat_half must not be NULL");
  const int ns = params->model == FSIB_NAVIER_STOKES ? 1 : 0;
  if (ns && !uhat_half) return fail(FSIB_ERR_ARG, "uhat_half must not be NULL for NAVIER_STOKES");
  const hipStream_t st = S(stream);
  if (ns) FSIB_TRY(dealiased_products(p, uhat_half, st));
  FSIB_HIP(fsib::launch_pressure(p, ns, params->rho, fhat_half, phat_half, st));
  return FSIB_OK;
}

fsib_status fsib_velocity(fsib_plan plan, const fsib_fluid_params* params, const fsib_force* force, int64_t M,
                          const double* X, void* U, void* uhat_half, void* stream) {
  if (!plan) return fail(FSIB_ERR_ARG, "plan is NULL");
  Plan& p = plan->p;
  FSIB_TRY(check_fluid(p, params));
  FSIB_TRY(check_points(p, M, X));
  FSIB_TRY(check_instances(p, M, force));
  if (M > 0 && !U) return fail(FSIB_ERR_ARG, "U is NULL");
  if (!uhat_half) return fail(FSIB_ERR_ARG, "uhat_half is NULL");
  if (params->model == FSIB_NAVIER_STOKES) {
    FSIB_HIP(fsib::launch_sort_points(p, M, X, S(stream)));
    return velocity_interp_sorted(p, M, uhat_half, U, S(stream));
  }
  FSIB_TRY(check_force(force, p.dim, M));
  return stokes_velocity(p, *params, *force, M, X, U, uhat_half, S(stream));
}

fsib_status fsib_step(fsib_plan plan, const fsib_fluid_params* params, const fsib_force* force, int64_t M, double* X,
                      void* U, void* uhat_half, double* diag, void* stream) {
  return fsib_steps(plan, params, force, M, X, U, uhat_half, 1, diag, stream);
}

fsib_status fsib_steps(fsib_plan plan, const fsib_fluid_params* params, const fsib_force* force, int64_t M, double* X,
                       void* U, void* uhat_half, int nsteps, double* diag, void* stream) {
  if (!plan) return fail(FSIB_ERR_ARG, "plan is NULL");
  Plan& p = plan->p;
  FSIB_TRY(check_fluid(p, params));
  FSIB_TRY(check_points(p, M, X));
  FSIB_TRY(check_force(force, p.dim, M));
  FSIB_TRY(check_instances(p, M, force));
  if (nsteps < 0) return fail(FSIB_ERR_ARG, "nsteps must be >= 0");
  if (p.ninst > 1 && diag) return fail(FSIB_ERR_ARG, "diag is not available on multi-instance plans");
  if (M > 0 && !U) return fail(FSIB_ERR_ARG, "U is NULL");
  if (!uhat_half) return fail(FSIB_ERR_ARG, "uhat_half is NULL");
  const hipStream_t st = S(stream);
  const fsib_fluid_params& prm = *params;
  const double dt = prm.dt;
  if (prm.model == FSIB_STOKES) {
    for (int n = 0; n < nsteps; ++n) {
      // X^{m+1/2} = X^m + dt/2 U^m (eq. spatial_1), then the midpoint rule with Stokes velocities
      FSIB_HIP(fsib::launch_axpy_positions(p, M, p.Xh, X, U, 0.5 * dt, st));
      FSIB_TRY(stokes_velocity(p, prm, *force, M, p.Xh, p.Uh, p.uhat_mid, st));
      FSIB_HIP(fsib::launch_axpy_positions(p, M, X, X, p.Uh, dt, st));
      FSIB_TRY(stokes_velocity(p, prm, *force, M, X, U, uhat_half, st));
    }
    if (diag && nsteps > 0) FSIB_HIP(fsib::launch_diag(p, prm, *force, M, p.F64, U, uhat_half, X, diag, st));
    return FSIB_OK;
  }
  const double Ld = p.dim == 3 ? p.L * p.L * p.L : p.L * p.L;
  // Each half step has a point side that no fluid work reads until the update: it runs on the plan's
  // second stream s2, forked from st after the work st holds and joined back before the update.  The
  // two sides touch disjoint buffers (the fine grid, its FFT buffers, fhat and the sorted points on
  // one side; the dealiasing buffers and the products on the other).  Between the steps of one call
  // the interpolation of U^{m+1} also stays on s2, beside the products of uhat^{m+1} that open the
  // next step (they do not read U); the last step joins it to st, so U is complete in st's order.
  const hipStream_t s2 = p.overlap && p.aux ? p.aux : st;
  // On an early error return the work already queued on s2 is joined to st as well, so that nothing
  // the caller may free or reuse next is still being written behind its back.
  struct JoinOnExit {
    hipStream_t st, s2;
    hipEvent_t ev;
    bool armed = false;
    ~JoinOnExit() {
      if (armed && s2 != st && hipEventRecord(ev, s2) == hipSuccess) (void)hipStreamWaitEvent(st, ev, 0);
    }
  } join{st, s2, p.fj[3]};
  if (nsteps > 0) {
    FSIB_HIP(hipEventRecord(p.fj[0], st));
    FSIB_HIP(hipStreamWaitEvent(s2, p.fj[0], 0));
    join.armed = true;
  }
  for (int n = 0; n < nsteps; ++n) {
    const bool last = n + 1 == nsteps;
    // X^{m+1/2} = X^m + dt/2 U^m (eq. spatial_1); F^{m+1/2} and fhat^{m+1/2} (eq. force_spreading_quad),
    // beside the products of uhat^m
    FSIB_HIP(fsib::launch_move_force_strengths(p, *force, M, p.Xh, X, U, 0.5 * dt, p.F64, p.S, s2));
    FSIB_HIP(fsib::launch_sort_points(p, M, p.Xh, s2, p.S));
    FSIB_TRY(force_spread_sorted(p, M, p.S, p.fhat, 1.0 / Ld, s2));
    FSIB_HIP(hipEventRecord(p.fj[1], s2));
    // uhat^{m+1/2} (eq. spatial_2), once fhat^{m+1/2} is complete
    FSIB_TRY(ns_update(p, fsib::FLUID_NS_HALF, prm, uhat_half, p.fhat, uhat_half, p.uhat_mid, p.fj[1], st, s2 != st));
    // U^{m+1/2} at X^{m+1/2} (points still sorted), X^{m+1} (eq. spatial_4) and its sort beside the
    // products of uhat^{m+1/2} and the full update (eq. spatial_3)
    FSIB_HIP(hipEventRecord(p.fj[2], st));
    FSIB_HIP(hipStreamWaitEvent(s2, p.fj[2], 0));
    FSIB_TRY(velocity_interp_sorted(p, M, p.uhat_mid, p.Uh, s2, X, dt));
    FSIB_HIP(fsib::launch_sort_points(p, M, X, s2));
    FSIB_TRY(ns_update(p, fsib::FLUID_NS_FULL, prm, p.uhat_mid, p.fhat, uhat_half, uhat_half, nullptr, st));
    // U^{m+1} at X^{m+1}: on s2 after the full update (the next step's products proceed on st), on st
    // after the last step
    if (last) {
      FSIB_HIP(hipEventRecord(p.fj[3], s2));
      FSIB_HIP(hipStreamWaitEvent(st, p.fj[3], 0));
      join.armed = false;
      FSIB_TRY(velocity_interp_sorted(p, M, uhat_half, U, st));
    } else {
      FSIB_HIP(hipEventRecord(p.fj[0], st));
      FSIB_HIP(hipStreamWaitEvent(s2, p.fj[0], 0));
      FSIB_TRY(velocity_interp_sorted(p, M, uhat_half, U, s2));
    }
  }
  if (diag && nsteps > 0) FSIB_HIP(fsib::launch_diag(p, prm, *force, M, p.F64, p.Uh, uhat_half, X, diag, st));
  return FSIB_OK;
}

fsib_status fsib_group_create(int nplans, const fsib_plan* plans, fsib_group* out) {
  if (!out) return fail(FSIB_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (nplans < 1 || nplans > fsib::kMaxParts) return fail(FSIB_ERR_ARG, "nplans must be in [1, 8]");
  if (!plans) return fail(FSIB_ERR_ARG, "plans is NULL");
  std::set<fsib_plan> seen;
  for (int g = 0; g < nplans; ++g) {
    if (!plans[g]) return fail(FSIB_ERR_ARG, "a plan of the group is NULL");
    if (!seen.insert(plans[g]).second) return fail(FSIB_ERR_ARG, "a plan appears twice in the group");
    const Plan& p = plans[g]->p;
    const Plan& p0 = plans[0]->p;
    if (!p.fluid || p.ns) return fail(FSIB_ERR_ARG, "group plans need fluid = 1 and navier_stokes = 0 (Stokes)");
    if (p.device != p0.device || p.dim != p0.dim || p.prec != p0.prec || p.w != p0.w || p.deg != p0.deg)
      return fail(FSIB_ERR_ARG, "group plans need one device, dimension, precision and kernel width");
  }
  fsib_group grp = new (std::nothrow) fsib_group_s;
  if (!grp) return fail(FSIB_ERR_OOM, "out of host memory");
  for (int g = 0; g < nplans; ++g) {
    grp->plans.push_back(plans[g]);
    grp->ps.push_back(&plans[g]->p);
  }
  *out = grp;
  return FSIB_OK;
}

fsib_status fsib_group_destroy(fsib_group group) {
  delete group;
  return FSIB_OK;
}

fsib_status fsib_group_steps(fsib_group group, const fsib_fluid_params* params, const fsib_force* forces,
                             const int64_t* M, double* const* X, void* const* U, void* const* uhat_half, int nsteps,
                             void* stream) {
  if (!group) return fail(FSIB_ERR_ARG, "group is NULL");
  if (!params || !forces || !M || !X || !U || !uhat_half) return fail(FSIB_ERR_ARG, "an operand array is NULL");
  if (nsteps < 0) return fail(FSIB_ERR_ARG, "nsteps must be >= 0");
  const std::vector<Plan*>& ps = group->ps;
  const size_t n = ps.size();
  for (size_t g = 0; g < n; ++g) {
    const Plan& p = *ps[g];
    FSIB_TRY(check_fluid(p, &params[g]));
    if (params[g].model != FSIB_STOKES) return fail(FSIB_ERR_ARG, "group steps take the Stokes model");
    FSIB_TRY(check_points(p, M[g], X[g]));
    FSIB_TRY(check_force(&forces[g], p.dim, M[g]));
    FSIB_TRY(check_instances(p, M[g], &forces[g]));
    if (M[g] > 0 && !U[g]) return fail(FSIB_ERR_ARG, "U is NULL");
    if (!uhat_half[g]) return fail(FSIB_ERR_ARG, "uhat_half is NULL");
  }
  const hipStream_t st = S(stream);
  std::vector<double*> Xh(n);
  std::vector<const double*> Xc(n), Xhc(n);
  std::vector<void*> Uh(n), umid(n);
  std::vector<const void*> Uc(n), Uhc(n);
  std::vector<double> half(n), full(n);
  for (size_t g = 0; g < n; ++g) {
    Xh[g] = ps[g]->Xh;
    Xhc[g] = ps[g]->Xh;
    Xc[g] = X[g];
    Uh[g] = ps[g]->Uh;
    Uhc[g] = ps[g]->Uh;
    Uc[g] = U[g];
    umid[g] = ps[g]->uhat_mid;
    half[g] = 0.5 * params[g].dt;
    full[g] = params[g].dt;
  }
  // The position updates ride on the interpolation passes: the one of U^{m+1/2} writes X^{m+1} = X^m +
  // dt U^{m+1/2}, the one of U^{m+1} writes the next step's X^{m+3/2} = X^{m+1} + dt/2 U^{m+1} (no
  // interpolation reads the positions it moves: it reads the sorted records).
  const fsib::GroupMove to_full{X, Xc.data(), full.data()};
  const fsib::GroupMove to_half{Xh.data(), Xc.data(), half.data()};
  for (int k = 0; k < nsteps; ++k) {
    // X^{m+1/2} = X^m + dt/2 U^m (eq. spatial_1), then the midpoint rule with Stokes velocities
    if (k == 0) FSIB_HIP(fsib::launch_axpy_positions_group(ps, M, Xh.data(), Xc.data(), Uc.data(), half.data(), st));
    FSIB_TRY(group_stokes_velocity(ps, params, forces, M, Xhc.data(), Uh.data(), umid.data(), st, &to_full));
    FSIB_TRY(group_stokes_velocity(ps, params, forces, M, Xc.data(), U, uhat_half, st,
                                   k + 1 < nsteps ? &to_half : nullptr));
  }
  return FSIB_OK;
}

}  // extern "C"
