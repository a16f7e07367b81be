// Host driver and C ABI of the ORAS-FGMRES Helmholtz library.
//
// Paper sec. 2.1 (right-preconditioned GMRES with the one-level ORAS
// preconditioner), sec. 2.2 (overlapping cuboids, local factorisations at
// set-up, forward/backward substitution on a block of right-hand sides,
// flexible GMRES), sec. 2.3 (27-point lambda-adaptive stencil), sec. 3.2
// (classical Gram-Schmidt, single vs double precision).
//
// Every entry point validates its arguments and the context state before
// touching the device, so a failing call leaves the context as it was.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "oras_internal.h"

namespace oras {
void fit_table(std::vector<double>& tab, double& g0, double& dg, int& count);
}

using namespace oras;

namespace {

struct Table {
  std::vector<double> w;
  double g0 = 0, dg = 0;
  int count = 0;
};

const Table& weight_table() {
  static Table t;
  static std::once_flag once;
  std::call_once(once, [] { fit_table(t.w, t.g0, t.dg, t.count); });
  return t;
}

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <typename T> T* as() const { return static_cast<T*>(p); }
};

}  // namespace

struct oras_ctx_s {
  int device = -1;
  hipStream_t stream = nullptr;
  // a second stream (and its fork/join events) for the factorisation, which
  // runs the two halves of the subdomains side by side
  hipStream_t stream2 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  bool host_only = true;
  std::string err;

  // operator
  bool assembled = false;
  int nx = 0, ny = 0, nz = 0;
  long long n = 0;
  double h = 0, omega = 0;
  int npml = 0, free_surface = 0;
  double c_ref = 0;
  int stencil_prec = ORAS_C128;
  DevBuf w7, mt, qf, px, py, pz, wtab, scratch8, gradw;
  // node fields of the matrix-free apply, per stencil precision; nodes
  // [mf_lo, mf_hi) per axis lie where every profile value they use is 1
  DevBuf mf4_64, mfim_64, mf4_32, mfim_32, mffac64, mffac32, mftiles;
  int mf_lo[3] = {0, 0, 0}, mf_hi[3] = {0, 0, 0};
  int mf_ntiles = 0, mf_nplain = 0;
  bool weights_match_m = false;   // the stencil weights are those of the current m
  double t_assemble = 0;

  // factors
  bool factored = false;
  int factor_prec = ORAS_C128;
  int parts[3] = {1, 1, 1};
  int overlap = 0;
  std::vector<SubDesc> subs;
  DevBuf subs_dev, fac, tbuf, lca, status, pstat;
  std::vector<double> pivot_ratio;          // min |pivot| / max |S_k| per subdomain plane
  double min_pivot_ratio = 0;
  int min_pivot_sub = -1, min_pivot_plane = -1;
  OrasPlan plan;
  int max_sz = 0, max_nt = 0;
  long long max_p = 0, max_box = 0, y_rows = 0, tv_rows = 0;
  double t_factor = 0;

  // block low-rank plane inverses (oras_compress_factors), dropped with the factors
  bool blr = false;
  DevBuf blr_bsubs, blr_items, blr_lists, blr_store, blr_bt;
  BlrApply blr_plan;
  long long blr_bt_rows = 0;
  std::vector<int> blr_ranks;               // per block, (sub, plane, I, J) order
  std::vector<long long> blr_rank_off;      // first block of (sub, plane): sub * max_sz + plane
  std::vector<int> blr_npch;
  std::vector<double> blr_f_fwd, blr_f_bwd, blr_b_fwd, blr_b_bwd;   // per plane step
  oras_blr_info blr_info{};

  // per-solve workspace (grown on demand)
  DevBuf ybuf, tvbuf, V, Z, Bint, Xint, Tmp, Tmp64, W32, partial, small;
  long long ws_s = 0;
  int ws_m = 0;

  // optional per-launch timing of the plane GEMM (HIP events on the stream)
  bool prof = false;
  std::vector<hipEvent_t> gemm_ev;
  std::vector<double> plane_p2_fwd, plane_p2_bwd, plane_p_fwd, plane_p_bwd;
  double gemm_s = 0, gemm_flops = 0, gemm_bytes = 0;
  double rhs_s = 0, rhs_bytes = 0;   // plane right-hand-side kernels (restriction fused)
  long long gemm_launches = 0;

  ~oras_ctx_s() {
    release_all();
    for (hipEvent_t e : gemm_ev) (void)hipEventDestroy(e);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (stream2) (void)hipStreamDestroy(stream2);
  }
  void release_blr() {
    blr_bsubs.release(); blr_items.release(); blr_lists.release(); blr_store.release();
    blr_bt.release();
    blr_plan = BlrApply();
    blr_ranks.clear();
    blr_rank_off.clear();
    blr_npch.clear();
    blr_bt_rows = 0;
    blr = false;
  }
  void release_factors() {
    release_blr();
    subs_dev.release(); fac.release(); tbuf.release(); lca.release();
    plan = OrasPlan();
    status.release();
    pstat.release();
    pivot_ratio.clear();
    min_pivot_ratio = 0;
    min_pivot_sub = min_pivot_plane = -1;
    ybuf.release(); tvbuf.release();
    subs.clear();
    factored = false;
  }
  void release_workspace() {
    V.release(); Z.release(); Bint.release(); Xint.release(); Tmp.release(); Tmp64.release();
    W32.release();
    partial.release(); small.release();
    ws_s = 0;
    ws_m = 0;
  }
  void release_all() {
    release_factors();
    release_workspace();
    w7.release(); mt.release(); qf.release(); px.release(); py.release(); pz.release();
    mf4_64.release(); mfim_64.release(); mf4_32.release(); mfim_32.release();
    mffac64.release(); mffac32.release(); mftiles.release();
    wtab.release(); scratch8.release(); gradw.release();
    assembled = false;
  }
};

namespace {

oras_status fail(oras_ctx c, oras_status st, const std::string& msg) {
  if (c) c->err = msg;
  return st;
}

#define HIP_TRY(ctx, expr)                                                         \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail(ctx, ORAS_E_HIP, std::string("HIP error ") + hipGetErrorString(e_) + \
                                       " at " #expr);                              \
  } while (0)

oras_status dev_alloc(oras_ctx c, DevBuf& b, size_t bytes) {
  if (b.bytes >= bytes && b.p) return ORAS_OK;
  b.release();
  if (bytes == 0) return ORAS_OK;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, ORAS_E_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  }
  b.p = p;
  b.bytes = bytes;
  return ORAS_OK;
}

#define TRY(expr)                        \
  do {                                   \
    oras_status s_ = (expr);             \
    if (s_ != ORAS_OK) return s_;        \
  } while (0)

oras_status check_device(oras_ctx c) {
  if (c->host_only) return fail(c, ORAS_E_HIP, "context has no device (created with device = -1)");
  HIP_TRY(c, hipSetDevice(c->device));
  return ORAS_OK;
}

oras_status check_free(oras_ctx c, double bytes) {
  size_t fr = 0, tot = 0;
  HIP_TRY(c, hipMemGetInfo(&fr, &tot));
  if (bytes > 0.97 * (double)fr)
    return fail(c, ORAS_E_OOM, "needs " + std::to_string(bytes / 1e9) + " GB, " +
                                   std::to_string((double)fr / 1e9) + " GB free");
  return ORAS_OK;
}

// Checks a model array on the device before the context changes: every one of
// its n entries must be finite and > 0.  max_out (may be null) receives the
// largest entry.
oras_status check_field(oras_ctx c, const double* x, long long n, const char* what,
                        double* max_out) {
  TRY(dev_alloc(c, c->scratch8, (size_t)field_check_doubles() * sizeof(double)));
  launch_field_check(x, n, c->scratch8.as<double>(), c->stream);
  double r[2] = {0.0, 0.0};
  HIP_TRY(c, hipMemcpyAsync(r, c->scratch8.p, sizeof(r), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (r[1] > 0.0)
    return fail(c, ORAS_E_ARG, std::string(what) + ": " + std::to_string((long long)r[1]) +
                                   " entries are not finite and > 0");
  if (max_out) *max_out = r[0];
  return ORAS_OK;
}

OpView opview(oras_ctx c) {
  OpView v;
  v.nx = c->nx;
  v.ny = c->ny;
  v.nz = c->nz;
  v.h = c->h;
  v.omega = c->omega;
  v.w7 = c->w7.as<double>();
  v.mt = c->mt.as<double2>();
  v.px = c->px.as<double2>();
  v.py = c->py.as<double2>();
  v.pz = c->pz.as<double2>();
  return v;
}

long long pad_s(int nrhs) { return ((long long)nrhs + RHS_ALIGN - 1) / RHS_ALIGN * RHS_ALIGN; }

size_t csize(int prec) { return prec == ORAS_C64 ? sizeof(float2) : sizeof(double2); }

// Nodes [lo, hi) of one axis whose profile values at offsets -1 .. 1 (half
// grid indices 2 i - 1 .. 2 i + 3, clamped as the apply clamps them) are
// exactly 1; lo = hi = 0 when they do not form one interval.
void plain_range(const std::vector<double2>& p, int n, int& lo, int& hi) {
  auto plain = [&](int i) {
    for (int t = 2 * i - 1; t <= 2 * i + 3; ++t) {
      const double2 v = p[std::min(std::max(t, 0), 2 * n)];
      if (v.x != 1.0 || v.y != 0.0) return false;
    }
    return true;
  };
  lo = 0;
  while (lo < n && !plain(lo)) ++lo;
  hi = lo;
  while (hi < n && plain(hi)) ++hi;
  for (int i = hi; i < n; ++i)
    if (plain(i)) { lo = hi = 0; return; }
  if (lo == hi) lo = hi = 0;
}

// Node fields of the matrix-free apply from w7 and m~ (both precisions the
// context applies A in: always FP64, for the true residual, and FP32 when the
// stencil runs in single precision), and the PML-free node ranges.
oras_status build_fields(oras_ctx c) {
  launch_mass_fields<double>(c->w7.as<double>(), c->mt.as<double2>(), c->n,
                             c->mf4_64.as<double4>(), c->mfim_64.as<double>(), c->stream);
  if (c->stencil_prec == ORAS_C64)
    launch_mass_fields<float>(c->w7.as<double>(), c->mt.as<double2>(), c->n,
                              c->mf4_32.as<float4>(), c->mfim_32.as<float>(), c->stream);
  HIP_TRY(c, hipGetLastError());
  // per-axis factor tables, 9 per node coordinate: R(d), H(d), N(d), d = -1, 0, 1
  const int ns[3] = {c->nx, c->ny, c->nz};
  const DevBuf* ps[3] = {&c->px, &c->py, &c->pz};
  std::vector<double2> fac64;
  for (int a = 0; a < 3; ++a) {
    std::vector<double2> p((size_t)(2 * ns[a] + 1));
    HIP_TRY(c, hipMemcpyAsync(p.data(), ps[a]->p, p.size() * sizeof(double2),
                              hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    plain_range(p, ns[a], c->mf_lo[a], c->mf_hi[a]);
    auto at = [&](int t) {
      const double2 v = p[std::min(std::max(t, 0), 2 * ns[a])];
      return std::complex<double>(v.x, v.y);
    };
    for (int i = 0; i < ns[a]; ++i) {
      const std::complex<double> hm = at(2 * i), hp = at(2 * i + 2);
      const std::complex<double> f[9] = {1.0 / hm, 1.0 / hm + 1.0 / hp, 1.0 / hp,
                                         hm, hm + hp, hp,
                                         at(2 * i - 1), at(2 * i + 1), at(2 * i + 3)};
      for (const auto& z : f) fac64.push_back(make_double2(z.real(), z.imag()));
    }
  }
  TRY(dev_alloc(c, c->mffac64, fac64.size() * sizeof(double2)));
  HIP_TRY(c, hipMemcpyAsync(c->mffac64.p, fac64.data(), fac64.size() * sizeof(double2),
                            hipMemcpyHostToDevice, c->stream));
  if (c->stencil_prec == ORAS_C64) {
    std::vector<float2> fac32(fac64.size());
    for (size_t i = 0; i < fac64.size(); ++i)
      fac32[i] = make_float2((float)fac64[i].x, (float)fac64[i].y);
    TRY(dev_alloc(c, c->mffac32, fac32.size() * sizeof(float2)));
    HIP_TRY(c, hipMemcpyAsync(c->mffac32.p, fac32.data(), fac32.size() * sizeof(float2),
                              hipMemcpyHostToDevice, c->stream));
  }
  std::vector<int> tiles;
  stencil_mf_tiles(c->mf_lo, c->mf_hi, c->nx, c->ny, c->nz, tiles, c->mf_nplain);
  c->mf_ntiles = (int)(tiles.size() / 4);
  TRY(dev_alloc(c, c->mftiles, tiles.size() * sizeof(int)));
  HIP_TRY(c, hipMemcpyAsync(c->mftiles.p, tiles.data(), tiles.size() * sizeof(int),
                            hipMemcpyHostToDevice, c->stream));
  // the host tables must outlive the copies
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return ORAS_OK;
}

template <typename R> StencilMF<R> mf_view(oras_ctx c);
template <> StencilMF<double> mf_view<double>(oras_ctx c) {
  StencilMF<double> v;
  v.f4 = c->mf4_64.as<double4>();
  v.fim = c->mfim_64.as<double>();
  v.fx = c->mffac64.as<double2>();
  return v;
}
template <> StencilMF<float> mf_view<float>(oras_ctx c) {
  StencilMF<float> v;
  v.f4 = c->mf4_32.as<float4>();
  v.fim = c->mfim_32.as<float>();
  v.fx = c->mffac32.as<float2>();
  return v;
}

// y (internal [n][s], c128 or, in single precision without b, c64) = A x, or
// b - A x when b is given, with x in the stencil precision R
template <typename R, typename Y = double2>
void apply_stencil(oras_ctx c, const C<R>* x, const double2* b, Y* y, int s, hipStream_t st) {
  StencilMF<R> v = mf_view<R>(c);
  v.fy = v.fx + 9 * c->nx;
  v.fz = v.fy + 9 * c->ny;
  v.tiles = c->mftiles.as<int4>();
  v.ntiles = c->mf_ntiles;
  v.nplain = c->mf_nplain;
  const Table& t = weight_table();
  const double ih2 = 1.0 / (c->h * c->h);
  // family weights (the same in every row of the table) with the averaging
  // factors of the in-plane (1/2 x 1/4) and cube-centre (1/16) differences
  v.W1 = t.w[0] * ih2;
  v.W2 = t.w[1] * ih2 * 0.125;
  v.W3 = t.w[2] * ih2 * 0.0625;
  v.om2 = c->omega * c->omega;
  launch_stencil_mf<R, Y>(v, x, b, y, c->nx, c->ny, c->nz, s, st);
}

int nblk_for(long long n) {
  long long b = (n + 255) / 256;
  return (int)std::max(1LL, std::min(2048LL, b));
}

// y (internal [n][s] c128) = A x in precision prec; x internal c128.
oras_status stencil_internal(oras_ctx c, const double2* x, const double2* b, double2* y, int s,
                             int prec) {
  if (prec == ORAS_C64) {
    TRY(dev_alloc(c, c->Tmp64, (size_t)c->n * s * sizeof(float2)));
    launch_cast<float>(x, c->Tmp64.as<float2>(), c->n * s, c->stream);
    apply_stencil<float>(c, c->Tmp64.as<float2>(), b, y, s, c->stream);
  } else {
    apply_stencil<double>(c, x, b, y, s, c->stream);
  }
  HIP_TRY(c, hipGetLastError());
  return ORAS_OK;
}

oras_status ensure_oras_ws(oras_ctx c, long long s) {
  const size_t cs = csize(c->factor_prec);
  TRY(dev_alloc(c, c->ybuf, (size_t)(c->y_rows * s) * cs));
  TRY(dev_alloc(c, c->tvbuf, plane_rhs_bytes(c->factor_prec, c->tv_rows, s)));
  return ORAS_OK;
}

// z (internal, factor precision or c128 when z128) = M^{-1} (scale * v)
oras_status oras_apply_internal(oras_ctx c, const double2* v, const double* scale, void* z, int s,
                                bool z128, int nrhs) {
  TRY(ensure_oras_ws(c, s));
  const int nsteps = 2 * c->max_sz - 1;
  // profiling: one event before the first plane step, then one after each
  // step's right-hand-side kernel and one after its products
  hipEvent_t* ev = nullptr;
  if (c->prof) {
    while ((int)c->gemm_ev.size() < 2 * nsteps + 1) {
      hipEvent_t e;
      HIP_TRY(c, hipEventCreate(&e));
      c->gemm_ev.push_back(e);
    }
    HIP_TRY(c, hipEventRecord(c->gemm_ev[0], c->stream));
    ev = c->gemm_ev.data() + 1;
  }
  const OrasPlan& pl = c->plan;
  if (c->blr) {
    const size_t cs = csize(c->factor_prec);
    // padding rows of the operand buffer must hold finite values (zero)
    const size_t bt_bytes = (size_t)(c->blr_bt_rows * pad16(s)) * cs;
    if (c->blr_bt.bytes < bt_bytes || !c->blr_bt.p) {
      TRY(dev_alloc(c, c->blr_bt, bt_bytes));
      launch_zero(c->blr_bt.p, c->blr_bt.bytes, c->stream);
    }
    const BlrApply& bp = c->blr_plan;
    if (c->factor_prec == ORAS_C64) {
      if (z128)
        launch_oras_apply_blr<float, double2>(bp, c->blr_store.as<float2>(), c->lca.as<float2>(),
                                              c->ybuf.as<float2>(), c->blr_bt.as<float2>(), v,
                                              scale, (double2*)z, c->nx, c->ny, s, c->stream, ev);
      else
        launch_oras_apply_blr<float, float2>(bp, c->blr_store.as<float2>(), c->lca.as<float2>(),
                                             c->ybuf.as<float2>(), c->blr_bt.as<float2>(), v,
                                             scale, (float2*)z, c->nx, c->ny, s, c->stream, ev);
    } else {
      launch_oras_apply_blr<double, double2>(bp, c->blr_store.as<double2>(),
                                             c->lca.as<double2>(), c->ybuf.as<double2>(),
                                             c->blr_bt.as<double2>(), v, scale, (double2*)z,
                                             c->nx, c->ny, s, c->stream, ev);
    }
  } else if (c->factor_prec == ORAS_C64) {
    if (z128)
      launch_oras_apply<float, double2>(pl, c->fac.as<float2>(), c->lca.as<float2>(),
                                        c->ybuf.as<float2>(), c->tvbuf.as<float2>(), v, scale,
                                        (double2*)z, c->nx, c->ny, s, c->stream, ev);
    else
      launch_oras_apply<float, float2>(pl, c->fac.as<float2>(), c->lca.as<float2>(),
                                       c->ybuf.as<float2>(), c->tvbuf.as<float2>(), v, scale,
                                       (float2*)z, c->nx, c->ny, s, c->stream, ev);
  } else {
    launch_oras_apply<double, double2>(pl, c->fac.as<double2>(), c->lca.as<double2>(),
                                       c->ybuf.as<double2>(), c->tvbuf.as<double2>(), v, scale,
                                       (double2*)z, c->nx, c->ny, s, c->stream, ev);
  }
  HIP_TRY(c, hipGetLastError());
  if (ev) {
    // per-launch durations and the algorithmic work of each plane step:
    // 8 p^2 nrhs flops; p^2 matrix entries + t read + y written (+ y read backward)
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const double cs = (double)csize(c->factor_prec);
    // right-hand side written: six bf16 pieces per FP32 complex value for the
    // dense products, the plain value otherwise
    const double tw = c->blr ? cs : (c->factor_prec == ORAS_C64 ? 12.0 : 16.0);
    for (int st = 0; st < nsteps; ++st) {
      float ms = 0, mr = 0;
      HIP_TRY(c, hipEventElapsedTime(&ms, ev[2 * st], ev[2 * st + 1]));
      HIP_TRY(c, hipEventElapsedTime(&mr, ev[2 * st - 1], ev[2 * st]));
      const bool bwd = st >= c->max_sz;
      const int k = bwd ? (c->max_sz - 2 - (st - c->max_sz)) : st;
      c->gemm_s += ms * 1e-3;
      c->gemm_launches += 1;
      // right-hand side of each active plane: v restricted (forward, FP64),
      // the neighbouring plane's y read (except forward plane 0), nine
      // couplings per row, t written
      {
        const double p1 = bwd ? c->plane_p_bwd[k] : c->plane_p_fwd[k];
        const bool couple = bwd || k > 0;
        c->rhs_s += mr * 1e-3;
        c->rhs_bytes += p1 * nrhs * ((bwd ? 0.0 : 16.0) + (couple ? cs : 0.0) + tw) +
                        (couple ? 9.0 * p1 * cs : 0.0);
      }
      if (c->blr) {
        // stored entries: 8 nrhs flops each; bytes: stored entries, gathered
        // rows and written rows (per right-hand side)
        c->gemm_flops += 8.0 * (bwd ? c->blr_f_bwd[k] : c->blr_f_fwd[k]) * nrhs;
        c->gemm_bytes += cs * ((bwd ? c->blr_f_bwd[k] : c->blr_f_fwd[k]) +
                               (bwd ? c->blr_b_bwd[k] : c->blr_b_fwd[k]) * nrhs);
        continue;
      }
      const double p2 = bwd ? c->plane_p2_bwd[k] : c->plane_p2_fwd[k];
      const double p1 = bwd ? c->plane_p_bwd[k] : c->plane_p_fwd[k];
      c->gemm_flops += 8.0 * p2 * nrhs;
      c->gemm_bytes += cs * (p2 + (bwd ? 3.0 : 2.0) * p1 * nrhs);
    }
  }
  return ORAS_OK;
}

double now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

// receiver indices live on the device: copy them back once and bound-check
oras_status check_receivers(oras_ctx c, const int* rec_dev, int nrec) {
  std::vector<int> r((size_t)nrec * 3);
  HIP_TRY(c, hipMemcpyAsync(r.data(), rec_dev, r.size() * sizeof(int), hipMemcpyDeviceToHost,
                            c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (int q = 0; q < nrec; ++q)
    if (r[3 * q] < 0 || r[3 * q] >= c->nx || r[3 * q + 1] < 0 || r[3 * q + 1] >= c->ny ||
        r[3 * q + 2] < 0 || r[3 * q + 2] >= c->nz)
      return fail(c, ORAS_E_ARG, "receiver index outside the grid");
  return ORAS_OK;
}

}  // namespace

// ------------------------------------------------------------------ C ABI --
namespace {

// Patch extents along one axis: n nodes in ceil(n / pmax) parts by floor split.
std::vector<int> patch_cuts(int n, int pmax) {
  const int parts = (n + pmax - 1) / pmax;
  std::vector<int> c(parts + 1);
  for (int t = 0; t <= parts; ++t) c[t] = (int)((long long)t * n / parts);
  return c;
}

struct TmpBufs {
  DevBuf smax, blocks, ranks, err;
  ~TmpBufs() { smax.release(); blocks.release(); ranks.release(); err.release(); }
};

// Items of one plane ordered so that item i runs on XCD i % 8 and every
// subdomain's items share an XCD (padding items have sub = -1).
void interleave(const std::vector<BlrItem>& in, std::vector<BlrItem>& out, int& first, int& count) {
  std::vector<std::vector<BlrItem>> bucket(8);
  for (const BlrItem& it : in) bucket[it.sub % 8].push_back(it);
  size_t longest = 0;
  for (auto& b : bucket) longest = std::max(longest, b.size());
  first = (int)out.size();
  BlrItem pad;
  std::memset(&pad, 0, sizeof(pad));
  pad.sub = -1;
  for (size_t i = 0; i < longest; ++i)
    for (int x = 0; x < 8; ++x) out.push_back(i < bucket[x].size() ? bucket[x][i] : pad);
  count = (int)(out.size() - first);
}

}  // namespace

namespace oras {

oras_status check_apply_A(oras_ctx c, const void* x_dev, const void* y_dev, int nrhs, int prec) {
  if (!c) return ORAS_E_ARG;
  if (!x_dev || !y_dev) return fail(c, ORAS_E_ARG, "null vector");
  if (nrhs < 1 || nrhs > 256) return fail(c, ORAS_E_ARG, "nrhs must be 1..256");
  if (prec != ORAS_C64 && prec != ORAS_C128) return fail(c, ORAS_E_ARG, "bad precision");
  if (!c->assembled) return fail(c, ORAS_E_STATE, "apply_A before assemble");
  if (prec == ORAS_C64 && c->stencil_prec != ORAS_C64)
    return fail(c, ORAS_E_STATE, "no complex64 stencil assembled");
  return check_device(c);
}

size_t apply_A_scratch_bytes(oras_ctx c, int nrhs, int prec) {
  const size_t ns = (size_t)(c->n * pad_s(nrhs));
  return ns * (2 * sizeof(double2) + (prec == ORAS_C64 ? sizeof(float2) : 0));
}

oras_status apply_A_staged(oras_ctx c, const void* x_dev, void* y_dev, int nrhs, int prec,
                           double2* xin, double2* yout, float2* x32) {
  const long long s = pad_s(nrhs);
  launch_to_internal((const double2*)x_dev, xin, c->n, nrhs, (int)s, 0, c->stream);
  if (prec == ORAS_C64) {
    launch_cast<float>(xin, x32, c->n * s, c->stream);
    apply_stencil<float>(c, x32, nullptr, yout, (int)s, c->stream);
  } else {
    apply_stencil<double>(c, xin, nullptr, yout, (int)s, c->stream);
  }
  launch_from_internal(yout, (double2*)y_dev, c->n, nrhs, (int)s, 0, c->stream);
  HIP_TRY(c, hipGetLastError());
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return ORAS_OK;
}

oras_status set_error(oras_ctx c, oras_status st, const char* msg) { return fail(c, st, msg); }

int ctx_device(oras_ctx c) { return c->device; }

}  // namespace oras

extern "C" {

oras_status oras_create(oras_ctx* out, int device, void* hip_stream) {
  if (!out) return ORAS_E_ARG;
  *out = nullptr;
  if (device < -1) return ORAS_E_ARG;
  oras_ctx c = new (std::nothrow) oras_ctx_s();
  if (!c) return ORAS_E_OOM;
  c->device = device;
  c->host_only = (device < 0);
  c->stream = (hipStream_t)hip_stream;
  if (!c->host_only) {
    int cnt = 0;
    if (hipGetDeviceCount(&cnt) != hipSuccess || device >= cnt) {
      (void)hipGetLastError();
      delete c;
      return ORAS_E_HIP;
    }
    if (hipSetDevice(device) != hipSuccess) {
      delete c;
      return ORAS_E_HIP;
    }
    // address of this device's copy of the no-alloc scratch (once per device;
    // a failure is kept and reported by the no-alloc entry point)
    oras::noalloc_init(device);
  }
  *out = c;
  return ORAS_OK;
}

void oras_destroy(oras_ctx ctx) {
  if (!ctx) return;
  if (!ctx->host_only) {
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
  }
  delete ctx;
}

const char* oras_last_error(oras_ctx ctx) {
  if (!ctx) return "null context";
  return ctx->err.c_str();
}

oras_status oras_weight_table(double* out_host, int capacity, double* g0, double* dg, int* count) {
  const Table& t = weight_table();
  if (count) *count = t.count;
  if (g0) *g0 = t.g0;
  if (dg) *dg = t.dg;
  if (!out_host) return ORAS_OK;
  if (capacity < t.count) return ORAS_E_ARG;
  std::memcpy(out_host, t.w.data(), sizeof(double) * 7 * t.count);
  return ORAS_OK;
}

oras_status oras_profile(oras_ctx ctx, int enable) {
  if (!ctx) return ORAS_E_ARG;
  ctx->prof = enable != 0;
  ctx->gemm_s = ctx->gemm_flops = ctx->gemm_bytes = 0;
  ctx->gemm_launches = 0;
  ctx->rhs_s = ctx->rhs_bytes = 0;
  return ORAS_OK;
}

oras_status oras_rhs_stats(oras_ctx ctx, double* seconds, double* bytes) {
  if (!ctx) return ORAS_E_ARG;
  if (seconds) *seconds = ctx->rhs_s;
  if (bytes) *bytes = ctx->rhs_bytes;
  return ORAS_OK;
}

oras_status oras_kernel_stats(oras_ctx ctx, double* gemm_seconds, long long* gemm_launches,
                              double* gemm_flops, double* gemm_bytes) {
  if (!ctx) return ORAS_E_ARG;
  if (gemm_seconds) *gemm_seconds = ctx->gemm_s;
  if (gemm_launches) *gemm_launches = ctx->gemm_launches;
  if (gemm_flops) *gemm_flops = ctx->gemm_flops;
  if (gemm_bytes) *gemm_bytes = ctx->gemm_bytes;
  return ORAS_OK;
}

oras_status oras_timings(oras_ctx ctx, double* t_assemble, double* t_factor) {
  if (!ctx) return ORAS_E_ARG;
  if (t_assemble) *t_assemble = ctx->t_assemble;
  if (t_factor) *t_factor = ctx->t_factor;
  return ORAS_OK;
}

oras_status oras_factor_stats(oras_ctx c, double* min_ratio, int* sub, int* plane,
                              double* ratios_host, int capacity, int* max_planes) {
  if (!c) return ORAS_E_ARG;
  if (!c->factored) return fail(c, ORAS_E_STATE, "factor_stats before factor_subdomains");
  if (min_ratio) *min_ratio = c->min_pivot_ratio;
  if (sub) *sub = c->min_pivot_sub;
  if (plane) *plane = c->min_pivot_plane;
  if (max_planes) *max_planes = c->max_sz;
  if (!ratios_host) return ORAS_OK;
  if (capacity < (long long)c->pivot_ratio.size())
    return fail(c, ORAS_E_ARG, "capacity below nsub * max_planes");
  std::memcpy(ratios_host, c->pivot_ratio.data(), c->pivot_ratio.size() * sizeof(double));
  return ORAS_OK;
}

oras_status oras_assemble(oras_ctx c, const oras_grid* g, const double* vel_dev,
                          const double* q_dev, double omega, const oras_pml* pml,
                          int stencil_prec) {
  if (!c) return ORAS_E_ARG;
  if (!g || !vel_dev || !pml) return fail(c, ORAS_E_ARG, "null grid, velocity or pml");
  if (g->nx < 3 || g->ny < 3 || g->nz < 3) return fail(c, ORAS_E_ARG, "grid needs >= 3 nodes per axis");
  if ((long long)g->nx * g->ny * g->nz > (1LL << 31))
    return fail(c, ORAS_E_OOM, "grid larger than 2^31 nodes");
  if (!finite_pos(g->h)) return fail(c, ORAS_E_ARG, "grid step must be finite and > 0");
  if (g->npml < 0 || 2 * g->npml >= std::min(g->nx, std::min(g->ny, g->nz)))
    return fail(c, ORAS_E_ARG, "npml must satisfy 0 <= 2 npml < min(nx, ny, nz)");
  if (!finite_pos(omega)) return fail(c, ORAS_E_ARG, "omega must be finite and > 0");
  if (!(pml->R0 > 0.0 && pml->R0 < 1.0)) return fail(c, ORAS_E_ARG, "pml R0 must be in (0, 1)");
  if (pml->power < 0 || pml->power > 8) return fail(c, ORAS_E_ARG, "pml power must be 0..8");
  if (!std::isfinite(pml->c_ref)) return fail(c, ORAS_E_ARG, "pml c_ref must be finite");
  if (stencil_prec != ORAS_C64 && stencil_prec != ORAS_C128)
    return fail(c, ORAS_E_ARG, "stencil_prec must be ORAS_C64 or ORAS_C128");
  TRY(check_device(c));
  const double t0 = now();
  const long long n = (long long)g->nx * g->ny * g->nz;
  // model checks first: a rejected model leaves the context as it was
  double vmax = 0;
  TRY(check_field(c, vel_dev, n, "velocity", &vmax));
  if (q_dev) TRY(check_field(c, q_dev, n, "Q", nullptr));
  const double need = (double)n * (7 * 8 + 16 * 2 + 40 + (stencil_prec == ORAS_C64 ? 20 : 0));
  {
    const double held = (double)(c->w7.bytes + c->mt.bytes + c->qf.bytes + c->mf4_64.bytes +
                                 c->mfim_64.bytes + c->mf4_32.bytes + c->mfim_32.bytes);
    TRY(check_free(c, need - held));
  }
  // buffers of an earlier assembly are reused when large enough; the factors
  // (and their compressed form) belong to the old operator
  c->assembled = false;
  c->release_blr();
  c->factored = false;
  c->nx = g->nx;
  c->ny = g->ny;
  c->nz = g->nz;
  c->n = n;
  c->h = g->h;
  c->omega = omega;
  c->npml = g->npml;
  c->free_surface = g->free_surface ? 1 : 0;
  c->stencil_prec = stencil_prec;
  const Table& t = weight_table();
  TRY(dev_alloc(c, c->w7, (size_t)n * 7 * sizeof(double)));
  TRY(dev_alloc(c, c->mt, (size_t)n * sizeof(double2)));
  TRY(dev_alloc(c, c->qf, (size_t)n * sizeof(double2)));
  TRY(dev_alloc(c, c->px, (size_t)(2 * g->nx + 1) * sizeof(double2)));
  TRY(dev_alloc(c, c->py, (size_t)(2 * g->ny + 1) * sizeof(double2)));
  TRY(dev_alloc(c, c->pz, (size_t)(2 * g->nz + 1) * sizeof(double2)));
  TRY(dev_alloc(c, c->mf4_64, (size_t)n * sizeof(double4)));
  TRY(dev_alloc(c, c->mfim_64, (size_t)n * sizeof(double)));
  if (stencil_prec == ORAS_C64) {
    TRY(dev_alloc(c, c->mf4_32, (size_t)n * sizeof(float4)));
    TRY(dev_alloc(c, c->mfim_32, (size_t)n * sizeof(float)));
  }
  TRY(dev_alloc(c, c->wtab, t.w.size() * sizeof(double)));
  HIP_TRY(c, hipMemcpyAsync(c->wtab.p, t.w.data(), t.w.size() * sizeof(double),
                            hipMemcpyHostToDevice, c->stream));
  c->c_ref = pml->c_ref > 0 ? pml->c_ref : vmax;
  launch_fields(vel_dev, q_dev, nullptr, c->wtab.as<double>(), t.count, t.g0, t.dg, c->nx, c->ny,
                c->nz, c->h, omega, c->w7.as<double>(), c->qf.as<double2>(), c->mt.as<double2>(),
                c->stream, 0);
  launch_pml(c->px.as<double2>(), c->nx, c->npml, c->h, omega, c->c_ref, pml->R0, pml->power, 1, 1,
             c->stream);
  launch_pml(c->py.as<double2>(), c->ny, c->npml, c->h, omega, c->c_ref, pml->R0, pml->power, 1, 1,
             c->stream);
  launch_pml(c->pz.as<double2>(), c->nz, c->npml, c->h, omega, c->c_ref, pml->R0, pml->power,
             c->free_surface ? 0 : 1, 1, c->stream);
  HIP_TRY(c, hipGetLastError());
  TRY(build_fields(c));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->assembled = true;
  c->weights_match_m = true;
  c->t_assemble = now() - t0;
  return ORAS_OK;
}

oras_status oras_set_m(oras_ctx c, const double* m_dev) { return oras_set_m_ex(c, m_dev, 0); }

oras_status oras_set_m_ex(oras_ctx c, const double* m_dev, int flags) {
  if (!c) return ORAS_E_ARG;
  if (!m_dev) return fail(c, ORAS_E_ARG, "null m");
  if (flags & ~ORAS_WEIGHTS_FOLLOW_M) return fail(c, ORAS_E_ARG, "unknown set_m flags");
  if (!c->assembled) return fail(c, ORAS_E_STATE, "set_m before assemble");
  TRY(check_device(c));
  TRY(check_field(c, m_dev, c->n, "m", nullptr));
  const Table& t = weight_table();
  c->release_factors();
  const bool follow = (flags & ORAS_WEIGHTS_FOLLOW_M) != 0;
  launch_fields(nullptr, nullptr, m_dev, c->wtab.as<double>(), t.count, t.g0, t.dg, c->nx, c->ny,
                c->nz, c->h, c->omega, c->w7.as<double>(), c->qf.as<double2>(), c->mt.as<double2>(),
                c->stream, follow ? 0 : 1);
  c->weights_match_m = follow;
  HIP_TRY(c, hipGetLastError());
  TRY(build_fields(c));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return ORAS_OK;
}

oras_status oras_factor_subdomains(oras_ctx c, const int parts[3], int overlap, int factor_prec) {
  return oras_factor_subdomains_ex(c, parts, overlap, factor_prec, nullptr);
}

oras_status oras_factor_subdomains_ex(oras_ctx c, const int parts[3], int overlap, int factor_prec,
                                      const oras_interface* iface) {
  if (!c) return ORAS_E_ARG;
  if (!parts) return fail(c, ORAS_E_ARG, "null parts");
  IfaceView ifc;
  ifc.kind = ORAS_IFACE_ROBIN;
  ifc.power = 2;
  ifc.R0 = 0.3;
  ifc.c_ref = 0.0;
  if (iface) {
    if (iface->kind != ORAS_IFACE_ROBIN && iface->kind != ORAS_IFACE_PML)
      return fail(c, ORAS_E_ARG, "interface kind must be ORAS_IFACE_ROBIN or ORAS_IFACE_PML");
    if (iface->kind == ORAS_IFACE_PML) {
      if (!(iface->R0 > 0.0 && iface->R0 < 1.0))
        return fail(c, ORAS_E_ARG, "interface PML R0 must lie in (0, 1)");
      if (iface->power < 1 || iface->power > 4)
        return fail(c, ORAS_E_ARG, "interface PML power must be 1..4");
      if (overlap < 1) return fail(c, ORAS_E_ARG, "PML interfaces need overlap >= 1");
      ifc.kind = ORAS_IFACE_PML;
      ifc.power = iface->power;
      ifc.R0 = iface->R0;
    }
  }
  if (factor_prec != ORAS_C64 && factor_prec != ORAS_C128)
    return fail(c, ORAS_E_ARG, "factor_prec must be ORAS_C64 or ORAS_C128");
  if (overlap < 0 || overlap > 8) return fail(c, ORAS_E_ARG, "overlap must be 0..8");
  for (int a = 0; a < 3; ++a)
    if (parts[a] < 1 || parts[a] > 256) return fail(c, ORAS_E_ARG, "parts must be 1..256");
  if (!c->assembled) return fail(c, ORAS_E_STATE, "factor_subdomains before assemble");
  const int nn[3] = {c->nx, c->ny, c->nz};
  for (int a = 0; a < 3; ++a)
    if (parts[a] > nn[a] / 2) return fail(c, ORAS_E_ARG, "partition finer than 2 nodes per part");

  // partition: floor split, overlap layers on interior sides (clipped)
  std::vector<SubDesc> subs;
  std::vector<int> cuts[3];
  for (int a = 0; a < 3; ++a)
    for (int t = 0; t <= parts[a]; ++t) cuts[a].push_back((int)(((long long)t * nn[a]) / parts[a]));
  long long fac_off = 0, lca_off = 0, y_rows = 0, t_off = 0, tv_rows = 0;
  int max_sz = 0, max_nt = 0;
  long long max_p = 0, max_box = 0;
  for (int tz = 0; tz < parts[2]; ++tz)
    for (int ty = 0; ty < parts[1]; ++ty)
      for (int tx = 0; tx < parts[0]; ++tx) {
        SubDesc d;
        std::memset(&d, 0, sizeof(d));
        const int tt[3] = {tx, ty, tz};
        for (int a = 0; a < 3; ++a) {
          d.olo[a] = cuts[a][tt[a]];
          d.ohi[a] = cuts[a][tt[a] + 1];
          d.lo[a] = std::max(0, d.olo[a] - overlap);
          d.hi[a] = std::min(nn[a], d.ohi[a] + overlap);
        }
        d.sx = d.hi[0] - d.lo[0];
        d.sy = d.hi[1] - d.lo[1];
        d.sz = d.hi[2] - d.lo[2];
        if (d.sx < 2 || d.sy < 2 || d.sz < 2)
          return fail(c, ORAS_E_ARG, "subdomain box thinner than 2 nodes");
        d.p = d.sx * d.sy;
        d.P = (d.p + TILE - 1) / TILE * TILE;
        d.nt = d.P / TILE;
        if (d.P > 8192) return fail(c, ORAS_E_ARG, "subdomain plane larger than 8192 nodes");
        d.fac_off = fac_off;
        d.lca_off = lca_off;
        d.y_off = y_rows;
        d.t_off = t_off;
        d.tv_off = tv_rows;
        fac_off += (long long)d.sz * d.P * d.P;
        lca_off += 27LL * d.sx * d.sy * d.sz;
        y_rows += (long long)d.sz * d.P;
        t_off += (long long)d.P * d.P;
        tv_rows += d.P;
        max_sz = std::max(max_sz, d.sz);
        max_nt = std::max(max_nt, d.nt);
        max_p = std::max(max_p, (long long)d.P);
        max_box = std::max(max_box, (long long)d.sx * d.sy * d.sz);
        subs.push_back(d);
      }
  const size_t cs = csize(factor_prec);
  const double need = (double)(fac_off + t_off + lca_off) * cs;
  TRY(check_device(c));
  {
    const double held = (double)(c->fac.bytes + c->tbuf.bytes + c->lca.bytes);
    TRY(check_free(c, need - held));
  }
  // the old factors (and their compressed form) are dropped from here on; the
  // buffers are reused when large enough
  c->release_blr();
  c->factored = false;
  DevBuf& tbuf = c->tbuf;
  TRY(dev_alloc(c, c->fac, (size_t)fac_off * cs));
  oras_status st = dev_alloc(c, tbuf, (size_t)t_off * cs);
  if (st != ORAS_OK) { c->release_factors(); return st; }
  TRY(dev_alloc(c, c->lca, (size_t)lca_off * cs));
  TRY(dev_alloc(c, c->subs_dev, subs.size() * sizeof(SubDesc)));
  TRY(dev_alloc(c, c->status, subs.size() * sizeof(int)));
  const size_t nstat = 2 * subs.size() * (size_t)max_sz;
  TRY(dev_alloc(c, c->pstat, nstat * sizeof(unsigned long long)));
  HIP_TRY(c, hipMemcpyAsync(c->subs_dev.p, subs.data(), subs.size() * sizeof(SubDesc),
                            hipMemcpyHostToDevice, c->stream));
  launch_zero(c->status.p, subs.size() * sizeof(int), c->stream);
  launch_zero(c->pstat.p, nstat * sizeof(unsigned long long), c->stream);
  const double t0 = now();
  ifc.c_ref = c->c_ref;
  launch_assemble_local(opview(c), c->subs_dev.as<SubDesc>(), (int)subs.size(), max_box, c->lca.p,
                        factor_prec, ifc, c->stream);
  HIP_TRY(c, hipGetLastError());
  // The subdomains are independent: two halves run their plane recursions on
  // two streams, so that one half's latency-bound kernels (the diagonal-block
  // inversions) overlap the other half's products.
  const int nsub = (int)subs.size();
  const int nh = nsub >= 16 ? nsub / 16 * 8 : nsub;
  const int nparts = nh < nsub ? 2 : 1;
  if (nparts == 2) {
    if (!c->stream2) HIP_TRY(c, hipStreamCreateWithFlags(&c->stream2, hipStreamNonBlocking));
    if (!c->ev_fork) HIP_TRY(c, hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
    if (!c->ev_join) HIP_TRY(c, hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
    HIP_TRY(c, hipEventRecord(c->ev_fork, c->stream));
    HIP_TRY(c, hipStreamWaitEvent(c->stream2, c->ev_fork, 0));
  }
  for (int part = 0; part < nparts; ++part) {
    const int s0 = part == 0 ? 0 : nh, ns = part == 0 ? nh : nsub - nh;
    hipStream_t st = part == 0 ? c->stream : c->stream2;
    const SubDesc* sd = c->subs_dev.as<SubDesc>() + s0;
    int* status = c->status.as<int>() + s0;
    unsigned long long* pstat = c->pstat.as<unsigned long long>() + 2 * (size_t)s0 * max_sz;
    for (int k = 0; k < max_sz; ++k) {
      if (factor_prec == ORAS_C64)
        launch_factor_plane<float>(sd, ns, k, max_nt, max_sz, c->fac.as<float2>(),
                                   tbuf.as<float2>(), c->lca.as<float2>(), status, pstat, st);
      else
        launch_factor_plane<double>(sd, ns, k, max_nt, max_sz, c->fac.as<double2>(),
                                    tbuf.as<double2>(), c->lca.as<double2>(), status, pstat, st);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) {
        c->release_factors();
        return fail(c, ORAS_E_HIP, std::string("factor launch: ") + hipGetErrorString(e));
      }
    }
  }
  if (nparts == 2) {
    HIP_TRY(c, hipEventRecord(c->ev_join, c->stream2));
    HIP_TRY(c, hipStreamWaitEvent(c->stream, c->ev_join, 0));
  }
  std::vector<int> stat(subs.size(), 0);
  std::vector<unsigned long long> pst(nstat, 0);
  HIP_TRY(c, hipMemcpyAsync(stat.data(), c->status.p, stat.size() * sizeof(int),
                            hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(pst.data(), c->pstat.p, nstat * sizeof(unsigned long long),
                            hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->t_factor = now() - t0;
  for (size_t j = 0; j < stat.size(); ++j)
    if (stat[j]) {
      c->release_factors();
      return fail(c, ORAS_E_NUMERIC,
                  "zero or non-finite pivot while factoring subdomain " + std::to_string(j));
    }
  // min |pivot| / max |S_k| per subdomain plane (NaN beyond a box's planes)
  c->pivot_ratio.assign(subs.size() * (size_t)max_sz, std::nan(""));
  c->min_pivot_ratio = INFINITY;
  for (size_t j = 0; j < subs.size(); ++j)
    for (int k = 0; k < subs[j].sz; ++k) {
      const size_t q = j * max_sz + k;
      double smax2, inv2;
      std::memcpy(&smax2, &pst[2 * q], sizeof(double));
      std::memcpy(&inv2, &pst[2 * q + 1], sizeof(double));
      const double r = (smax2 > 0 && inv2 > 0) ? 1.0 / std::sqrt(smax2 * inv2) : 0.0;
      c->pivot_ratio[q] = r;
      if (r < c->min_pivot_ratio) {
        c->min_pivot_ratio = r;
        c->min_pivot_sub = (int)j;
        c->min_pivot_plane = k;
      }
    }
  c->plane_p2_fwd.assign(max_sz, 0.0);
  c->plane_p2_bwd.assign(max_sz, 0.0);
  c->plane_p_fwd.assign(max_sz, 0.0);
  c->plane_p_bwd.assign(max_sz, 0.0);
  for (const SubDesc& d : subs)
    for (int k = 0; k < d.sz; ++k) {
      c->plane_p2_fwd[k] += (double)d.p * d.p;
      c->plane_p_fwd[k] += d.p;
      if (k <= d.sz - 2 && k >= d.olo[2] - d.lo[2]) {   // backward planes that feed the output
        c->plane_p2_bwd[k] += (double)d.p * d.p;
        c->plane_p_bwd[k] += d.p;
      }
    }
  c->subs = subs;
  c->factor_prec = factor_prec;
  c->parts[0] = parts[0];
  c->parts[1] = parts[1];
  c->parts[2] = parts[2];
  c->overlap = overlap;
  c->max_sz = max_sz;
  c->max_nt = max_nt;
  c->max_p = max_p;
  c->max_box = max_box;
  c->y_rows = y_rows;
  c->tv_rows = tv_rows;
  c->plan.subs = c->subs_dev.as<SubDesc>();
  c->plan.nsub = (int)subs.size();
  c->plan.max_sz = max_sz;
  c->plan.max_nt = max_nt;
  c->plan.max_p = max_p;
  c->factored = true;
  return ORAS_OK;
}

oras_status oras_compress_factors(oras_ctx c, double eps, int pmax, oras_blr_info* info) {
  if (!c) return ORAS_E_ARG;
  if (!(eps >= 0.0 && eps < 1.0)) return fail(c, ORAS_E_ARG, "eps must lie in [0, 1)");
  if (pmax < 2 || pmax > BLR_PMAX) return fail(c, ORAS_E_ARG, "pmax must be 2..8");
  if (!c->factored) return fail(c, ORAS_E_STATE, "compress_factors before factor_subdomains");
  TRY(check_device(c));
  c->release_blr();
  const double t0 = now();
  const int nsub = (int)c->subs.size(), max_sz = c->max_sz;
  const size_t cs = csize(c->factor_prec);
  std::vector<BlrSub> bsubs(nsub);
  std::vector<std::vector<int>> cx(nsub), cy(nsub);
  std::vector<int> npch(nsub);
  std::vector<long long> rank_off((size_t)nsub * max_sz, -1);
  long long nblocks = 0;
  for (int j = 0; j < nsub; ++j) {
    const SubDesc& d = c->subs[j];
    cx[j] = patch_cuts(d.sx, pmax);
    cy[j] = patch_cuts(d.sy, pmax);
    bsubs[j].npx = (int)cx[j].size() - 1;
    bsubs[j].npy = (int)cy[j].size() - 1;
    bsubs[j].bt_off = 0;
    npch[j] = bsubs[j].npx * bsubs[j].npy;
    for (int k = 0; k < d.sz; ++k) {
      rank_off[(size_t)j * max_sz + k] = nblocks;
      nblocks += (long long)npch[j] * npch[j];
    }
  }
  if (nblocks >= (1LL << 31)) return fail(c, ORAS_E_ARG, "too many patch blocks");
  std::vector<BlrBlock> blocks((size_t)nblocks);
  for (int j = 0; j < nsub; ++j)
    for (int k = 0; k < c->subs[j].sz; ++k) {
      long long b = rank_off[(size_t)j * max_sz + k];
      for (int I = 0; I < npch[j]; ++I)
        for (int J = 0; J < npch[j]; ++J, ++b) {
          BlrBlock& x = blocks[(size_t)b];
          std::memset(&x, 0, sizeof(x));
          x.sub = j;
          x.k = k;
          x.I = I;
          x.J = J;
          x.rank = -1;
          x.p_off = -1;
        }
    }
  // pass 1: ranks
  TmpBufs tmp;
  TRY(check_free(c, (double)nblocks * (sizeof(BlrBlock) + sizeof(int)) + 8.0 * nsub * max_sz));
  TRY(dev_alloc(c, tmp.smax, (size_t)nsub * max_sz * sizeof(double)));
  TRY(dev_alloc(c, tmp.blocks, (size_t)nblocks * sizeof(BlrBlock)));
  TRY(dev_alloc(c, tmp.ranks, (size_t)nblocks * sizeof(int)));
  TRY(dev_alloc(c, tmp.err, sizeof(int)));
  TRY(dev_alloc(c, c->blr_bsubs, (size_t)nsub * sizeof(BlrSub)));
  HIP_TRY(c, hipMemcpyAsync(c->blr_bsubs.p, bsubs.data(), (size_t)nsub * sizeof(BlrSub),
                            hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(tmp.blocks.p, blocks.data(), (size_t)nblocks * sizeof(BlrBlock),
                            hipMemcpyHostToDevice, c->stream));
  const SubDesc* sdev = c->subs_dev.as<SubDesc>();
  if (c->factor_prec == ORAS_C64) {
    launch_blr_plane_max<float>(sdev, nsub, max_sz, c->fac.as<float2>(), tmp.smax.as<double>(),
                                c->stream);
    launch_blr_compress<float>(sdev, c->blr_bsubs.as<BlrSub>(), tmp.blocks.as<BlrBlock>(), nblocks,
                               c->fac.as<float2>(), tmp.smax.as<double>(), max_sz, eps,
                               tmp.ranks.as<int>(), nullptr, nullptr, c->stream);
  } else {
    launch_blr_plane_max<double>(sdev, nsub, max_sz, c->fac.as<double2>(), tmp.smax.as<double>(),
                                 c->stream);
    launch_blr_compress<double>(sdev, c->blr_bsubs.as<BlrSub>(), tmp.blocks.as<BlrBlock>(),
                                nblocks, c->fac.as<double2>(), tmp.smax.as<double>(), max_sz, eps,
                                tmp.ranks.as<int>(), nullptr, nullptr, c->stream);
  }
  HIP_TRY(c, hipGetLastError());
  std::vector<int> ranks((size_t)nblocks);
  HIP_TRY(c, hipMemcpyAsync(ranks.data(), tmp.ranks.p, (size_t)nblocks * sizeof(int),
                            hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));

  // layout: per subdomain the t rows (patch-major, each patch padded to a
  // multiple of 8 rows), then per plane the T rows of every row patch I
  // (T_I = [T_IJ for the low-rank blocks, J ascending], padded likewise)
  std::vector<std::vector<BlrItem>> pit(max_sz), eit(max_sz);
  std::vector<int> lists;
  long long store = 0;
  std::vector<long long> tcap(nsub, 0), trows(nsub, 0);
  std::vector<double> f_fwd(max_sz, 0.0), f_bwd(max_sz, 0.0), b_fwd(max_sz, 0.0),
      b_bwd(max_sz, 0.0);
  oras_blr_info inf{};
  inf.eps = eps;
  inf.pmax = pmax;
  double rank_sum = 0;
  // runs of operand rows come in whole pairs of 4-row groups (multiples of 8)
  auto pad8 = [](int v) { return (v + 7) / 8 * 8; };
  for (int j = 0; j < nsub; ++j) {
    const SubDesc& d = c->subs[j];
    const int np = npch[j], npx = bsubs[j].npx;
    std::vector<int> bsz(np), toff(np);
    bsubs[j].ptab = (int)lists.size();
    int tt = 0;
    for (int I = 0; I < np; ++I) {
      const int px = I % npx, py = I / npx;
      bsz[I] = (cx[j][px + 1] - cx[j][px]) * (cy[j][py + 1] - cy[j][py]);
      toff[I] = tt;
      lists.push_back(tt);
      tt += pad8(bsz[I]);
    }
    trows[j] = tt;
    for (int k = 0; k < d.sz; ++k) {
      const long long base = rank_off[(size_t)j * max_sz + k];
      auto rk = [&](int I, int J) { return ranks[(size_t)(base + (long long)I * np + J)]; };
      const bool act_bwd = k <= d.sz - 2 && k >= d.olo[2] - d.lo[2];
      double fl = 0, by = 0;
      // T rows of every row patch
      std::vector<int> RI(np, 0), toffT(np, 0), offIJ((size_t)np * np, 0);
      int trow = tt;
      for (int I = 0; I < np; ++I) {
        for (int J = 0; J < np; ++J)
          if (J != I && rk(I, J) >= 0) {
            offIJ[(size_t)I * np + J] = RI[I];
            RI[I] += rk(I, J);
          }
        toffT[I] = trow;
        trow += pad8(RI[I]);
      }
      tcap[j] = std::max(tcap[j], (long long)(trow - tt));
      // projection operands: V of the low-rank blocks of column patch J, stacked by I
      std::vector<int> prow((size_t)np * np, 0), pmp(np, 0);
      std::vector<long long> poff(np, -1);
      for (int J = 0; J < np; ++J) {
        int RJ = 0;
        for (int I = 0; I < np; ++I)
          if (I != J && rk(I, J) >= 0) {
            prow[(size_t)I * np + J] = RJ;
            RJ += rk(I, J);
          }
        if (RJ == 0) continue;
        const int mp = (RJ + 31) / 32 * 32, kp = pad8(bsz[J]);
        poff[J] = store;
        pmp[J] = mp;
        std::vector<int> dest(mp, 0);
        for (int I = 0; I < np; ++I)
          if (I != J && rk(I, J) >= 0)
            for (int q = 0; q < rk(I, J); ++q)
              dest[prow[(size_t)I * np + J] + q] = toffT[I] + offIJ[(size_t)I * np + J] + q;
        for (int rt = 0; rt < mp / 32; ++rt) {
          BlrItem it;
          std::memset(&it, 0, sizeof(it));
          it.sub = j;
          it.patch = J;
          it.rows = std::min(32, RJ - 32 * rt);
          it.mpad = mp;
          it.K = kp;
          it.row0 = 32 * rt;
          it.brow = toff[J];
          it.a_off = store;
          it.list_off = (long long)lists.size();
          lists.insert(lists.end(), dest.begin() + 32 * rt, dest.begin() + 32 * rt + 32);
          pit[k].push_back(it);
        }
        store += (long long)mp * kp;
        fl += (double)RJ * bsz[J];
        by += bsz[J] + RJ;
      }
      // expansion operands: [S_II | S_IJ dense | U_IJ low-rank] of row patch I
      for (int I = 0; I < np; ++I) {
        while (lists.size() % 4) lists.push_back(0);     // int4 segments
        const long long loff = (long long)lists.size();
        std::vector<int> koff(np, 0);
        int K = 0, nseg = 0, kd = 0;
        auto seg = [&](int row, int len) {
          lists.push_back(K);
          lists.push_back(row);
          lists.push_back(len);
          lists.push_back(0);
          K += len;
          ++nseg;
        };
        seg(toff[I], pad8(bsz[I]));
        kd += bsz[I];
        for (int J = 0; J < np; ++J)
          if (J != I && rk(I, J) < 0) {
            koff[J] = K;
            seg(toff[J], pad8(bsz[J]));
            kd += bsz[J];
          }
        const int kT = K;
        if (RI[I] > 0) seg(toffT[I], pad8(RI[I]));
        for (int J = 0; J < np; ++J)
          if (J != I && rk(I, J) >= 0) koff[J] = kT + offIJ[(size_t)I * np + J];
        BlrItem it;
        std::memset(&it, 0, sizeof(it));
        it.sub = j;
        it.patch = I;
        it.rows = bsz[I];
        it.mpad = 64;
        it.K = K;
        it.nseg = nseg;
        it.a_off = store;
        it.list_off = loff;
        if (bsz[I] > 32) {
          // the expansion runs 32 rows per wave: two items per patch
          BlrItem it2 = it;
          it.rows = 32;
          it2.row0 = 32;
          it2.rows = bsz[I] - 32;
          eit[k].push_back(it);
          eit[k].push_back(it2);
        } else {
          eit[k].push_back(it);
        }
        for (int J = 0; J < np; ++J) {
          BlrBlock& x = blocks[(size_t)(base + (long long)I * np + J)];
          x.rank = J == I ? -1 : rk(I, J);
          x.e_off = store;
          x.e_koff = koff[J];
          if (J != I && x.rank >= 0) {
            x.p_off = poff[J];
            x.p_mpad = pmp[J];
            x.p_row = prow[(size_t)I * np + J];
            inf.lowrank += 1;
            rank_sum += x.rank;
            inf.max_rank = std::max(inf.max_rank, x.rank);
          }
          if (J != I) inf.blocks += 1;
        }
        store += 64LL * K;
        fl += (double)bsz[I] * (kd + RI[I]);
        by += kd + RI[I] + (act_bwd ? 2.0 : 1.0) * bsz[I];
      }
      f_fwd[k] += fl;
      b_fwd[k] += by;
      if (act_bwd) {
        f_bwd[k] += fl;
        b_bwd[k] += by;
      }
      inf.stored_entries += fl;
      inf.dense_entries += (double)d.p * d.p;
    }
  }
  inf.mean_rank = inf.lowrank ? rank_sum / inf.lowrank : 0.0;
  long long bt_rows = 0;
  for (int j = 0; j < nsub; ++j) {
    bsubs[j].bt_off = bt_rows;
    bt_rows += trows[j] + tcap[j];
  }
  std::vector<BlrItem> items;
  BlrApply& pl = c->blr_plan;
  pl.p_first.assign(max_sz, 0);
  pl.p_count.assign(max_sz, 0);
  pl.e_first.assign(max_sz, 0);
  pl.e_count.assign(max_sz, 0);
  for (int k = 0; k < max_sz; ++k) {
    interleave(pit[k], items, pl.p_first[k], pl.p_count[k]);
    interleave(eit[k], items, pl.e_first[k], pl.e_count[k]);
  }
  // pass 2: write the operands
  TRY(check_free(c, (double)store * cs + (double)items.size() * sizeof(BlrItem) +
                        (double)lists.size() * sizeof(int)));
  TRY(dev_alloc(c, c->blr_store, (size_t)std::max(store, 1LL) * cs));
  TRY(dev_alloc(c, c->blr_items, std::max<size_t>(items.size(), 1) * sizeof(BlrItem)));
  TRY(dev_alloc(c, c->blr_lists, std::max<size_t>(lists.size(), 1) * sizeof(int)));
  launch_zero(c->blr_store.p, (size_t)store * cs, c->stream);
  launch_zero(tmp.err.p, sizeof(int), c->stream);
  HIP_TRY(c, hipMemcpyAsync(c->blr_bsubs.p, bsubs.data(), (size_t)nsub * sizeof(BlrSub),
                            hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(tmp.blocks.p, blocks.data(), (size_t)nblocks * sizeof(BlrBlock),
                            hipMemcpyHostToDevice, c->stream));
  if (!items.empty())
    HIP_TRY(c, hipMemcpyAsync(c->blr_items.p, items.data(), items.size() * sizeof(BlrItem),
                              hipMemcpyHostToDevice, c->stream));
  if (!lists.empty())
    HIP_TRY(c, hipMemcpyAsync(c->blr_lists.p, lists.data(), lists.size() * sizeof(int),
                              hipMemcpyHostToDevice, c->stream));
  if (c->factor_prec == ORAS_C64)
    launch_blr_compress<float>(sdev, c->blr_bsubs.as<BlrSub>(), tmp.blocks.as<BlrBlock>(), nblocks,
                               c->fac.as<float2>(), tmp.smax.as<double>(), max_sz, eps, nullptr,
                               c->blr_store.as<float2>(), tmp.err.as<int>(), c->stream);
  else
    launch_blr_compress<double>(sdev, c->blr_bsubs.as<BlrSub>(), tmp.blocks.as<BlrBlock>(),
                                nblocks, c->fac.as<double2>(), tmp.smax.as<double>(), max_sz, eps,
                                nullptr, c->blr_store.as<double2>(), tmp.err.as<int>(), c->stream);
  HIP_TRY(c, hipGetLastError());
  int err = 0;
  HIP_TRY(c, hipMemcpyAsync(&err, tmp.err.p, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (err) {
    c->release_blr();
    return fail(c, ORAS_E_NUMERIC, "BLR compression did not reproduce its ranks");
  }
  pl.subs = sdev;
  pl.bsubs = c->blr_bsubs.as<BlrSub>();
  pl.items = c->blr_items.as<BlrItem>();
  pl.lists = c->blr_lists.as<int>();
  pl.nsub = nsub;
  pl.max_sz = max_sz;
  pl.max_p = c->max_p;
  c->blr_bt_rows = bt_rows;
  c->blr_ranks.swap(ranks);
  c->blr_rank_off.swap(rank_off);
  c->blr_npch.swap(npch);
  c->blr_f_fwd = f_fwd;
  c->blr_f_bwd = f_bwd;
  c->blr_b_fwd = b_fwd;
  c->blr_b_bwd = b_bwd;
  inf.t_compress = now() - t0;
  c->blr_info = inf;
  c->blr = true;
  if (info) *info = inf;
  return ORAS_OK;
}

oras_status oras_blr_ranks(oras_ctx c, int sub, int plane, int* ranks_host, int capacity,
                           int* npatch) {
  if (!c) return ORAS_E_ARG;
  if (!c->blr) return fail(c, ORAS_E_STATE, "no compressed factors");
  if (sub < 0 || sub >= (int)c->subs.size()) return fail(c, ORAS_E_ARG, "sub out of range");
  if (plane < 0 || plane >= c->subs[sub].sz) return fail(c, ORAS_E_ARG, "plane out of range");
  const int np = c->blr_npch[sub];
  if (npatch) *npatch = np;
  if (!ranks_host) return ORAS_OK;
  if (capacity < np * np) return fail(c, ORAS_E_ARG, "capacity below npatch^2");
  const long long base = c->blr_rank_off[(size_t)sub * c->max_sz + plane];
  for (int q = 0; q < np * np; ++q) ranks_host[q] = c->blr_ranks[(size_t)(base + q)];
  return ORAS_OK;
}

oras_status oras_subdomain(oras_ctx c, int j, int* nsub, int* box12) {
  if (!c) return ORAS_E_ARG;
  if (!c->factored) return fail(c, ORAS_E_STATE, "no factors");
  if (nsub) *nsub = (int)c->subs.size();
  if (!box12) return ORAS_OK;
  if (j < 0 || j >= (int)c->subs.size()) return fail(c, ORAS_E_ARG, "subdomain index out of range");
  const SubDesc& d = c->subs[j];
  for (int a = 0; a < 3; ++a) {
    box12[a] = d.lo[a];
    box12[3 + a] = d.hi[a];
    box12[6 + a] = d.olo[a];
    box12[9 + a] = d.ohi[a];
  }
  return ORAS_OK;
}

oras_status oras_apply_A(oras_ctx c, const void* x_dev, void* y_dev, int nrhs, int prec) {
  TRY(oras::check_apply_A(c, x_dev, y_dev, nrhs, prec));
  const long long s = pad_s(nrhs);
  TRY(dev_alloc(c, c->Bint, (size_t)(c->n * s) * sizeof(double2)));
  TRY(dev_alloc(c, c->Tmp, (size_t)(c->n * s) * sizeof(double2)));
  if (prec == ORAS_C64) TRY(dev_alloc(c, c->Tmp64, (size_t)(c->n * s) * sizeof(float2)));
  return oras::apply_A_staged(c, x_dev, y_dev, nrhs, prec, c->Bint.as<double2>(),
                              c->Tmp.as<double2>(),
                              prec == ORAS_C64 ? c->Tmp64.as<float2>() : nullptr);
}

oras_status oras_apply_M(oras_ctx c, const void* x_dev, void* y_dev, int nrhs) {
  if (!c) return ORAS_E_ARG;
  if (!x_dev || !y_dev) return fail(c, ORAS_E_ARG, "null vector");
  if (nrhs < 1 || nrhs > 256) return fail(c, ORAS_E_ARG, "nrhs must be 1..256");
  if (!c->factored) return fail(c, ORAS_E_STATE, "apply_M before factor_subdomains");
  TRY(check_device(c));
  const long long s = pad_s(nrhs);
  TRY(dev_alloc(c, c->Bint, (size_t)(c->n * s) * sizeof(double2)));
  TRY(dev_alloc(c, c->Tmp, (size_t)(c->n * s) * sizeof(double2)));
  launch_to_internal((const double2*)x_dev, c->Bint.as<double2>(), c->n, nrhs, (int)s, 0, c->stream);
  TRY(oras_apply_internal(c, c->Bint.as<double2>(), nullptr, c->Tmp.p, (int)s, true, nrhs));
  launch_from_internal(c->Tmp.as<double2>(), (double2*)y_dev, c->n, nrhs, (int)s, 0, c->stream);
  HIP_TRY(c, hipGetLastError());
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return ORAS_OK;
}

oras_status oras_coefficients(oras_ctx c, void* out_dev) {
  if (!c) return ORAS_E_ARG;
  if (!out_dev) return fail(c, ORAS_E_ARG, "null output");
  if (!c->assembled) return fail(c, ORAS_E_STATE, "coefficients before assemble");
  TRY(check_device(c));
  // assembled on demand: the apply itself forms them from the node fields
  launch_assemble_global(opview(c), (double2*)out_dev, c->stream);
  HIP_TRY(c, hipGetLastError());
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return ORAS_OK;
}

oras_status oras_solve(oras_ctx c, const void* b_dev, void* x_dev, int nrhs, double tol,
                       const oras_solve_opts* opts, oras_solve_info* info) {
  if (!c) return ORAS_E_ARG;
  if (!b_dev || !x_dev) return fail(c, ORAS_E_ARG, "null b or x");
  if (nrhs < 1 || nrhs > 256) return fail(c, ORAS_E_ARG, "nrhs must be 1..256");
  if (!(tol > 0.0 && tol < 1.0)) return fail(c, ORAS_E_ARG, "tol must be in (0, 1)");
  oras_solve_opts o = {30, 1000, 0, 0, 0};
  if (opts) o = *opts;
  if (o.restart < 1 || o.restart > 200) return fail(c, ORAS_E_ARG, "restart must be 1..200");
  if (o.maxit < 1) return fail(c, ORAS_E_ARG, "maxit must be >= 1");
  if (o.flags & ~(ORAS_CONJ | ORAS_X0)) return fail(c, ORAS_E_ARG, "unknown flags");
  auto prec_ok = [](int p) { return p == 0 || p == ORAS_C64 || p == ORAS_C128; };
  if (!prec_ok(o.krylov_in_prec)) return fail(c, ORAS_E_ARG, "krylov_in_prec must be 0, C64 or C128");
  if (!prec_ok(o.z_prec)) return fail(c, ORAS_E_ARG, "z_prec must be 0, C64 or C128");
  if (!c->assembled) return fail(c, ORAS_E_STATE, "solve before assemble");
  if (!c->factored) return fail(c, ORAS_E_STATE, "solve before factor_subdomains");
  if (c->stencil_prec != c->factor_prec)
    return fail(c, ORAS_E_ARG, "stencil and factor precisions must match");
  // precision of the product A z_j and of the stored basis Z
  const int kprec = o.krylov_in_prec ? o.krylov_in_prec : c->stencil_prec;
  const int zprec = o.z_prec ? o.z_prec : c->factor_prec;
  if (kprec == ORAS_C64 && c->stencil_prec != ORAS_C64)
    return fail(c, ORAS_E_ARG, "krylov_in_prec C64 needs a context assembled in C64");
  if (zprec == ORAS_C64 && c->factor_prec != ORAS_C64)
    return fail(c, ORAS_E_ARG, "z_prec C64 needs C64 factors");
  TRY(check_device(c));
  const double t0 = now();
  const hipStream_t st = c->stream;
  const int m = o.restart;
  const long long s = pad_s(nrhs);
  const long long n = c->n;
  const long long ns = n * s;
  const bool z64 = (zprec == ORAS_C64);
  const size_t zsz = z64 ? sizeof(float2) : sizeof(double2);
  // A z_j in another precision than Z is stored in goes through a converted copy
  const bool convert = (kprec == ORAS_C64) != z64;
  const int nblk = nblk_for(n);
  {
    double need = 0;
    if (!c->V.p || c->ws_s < s || c->ws_m < m) need += (double)ns * ((m + 1) * 16.0 + m * zsz + 2 * 16.0);
    if (kprec == ORAS_C64 && c->W32.bytes < (size_t)ns * sizeof(float2)) need += (double)ns * 8.0;
    if (convert) {
      const DevBuf& tb = kprec == ORAS_C64 ? c->Tmp64 : c->Tmp;
      const size_t tbytes = (size_t)ns * (kprec == ORAS_C64 ? sizeof(float2) : sizeof(double2));
      if (tb.bytes < tbytes) need += (double)tbytes;
    }
    TRY(check_free(c, need));
  }
  if (convert) {
    if (kprec == ORAS_C64) TRY(dev_alloc(c, c->Tmp64, (size_t)ns * sizeof(float2)));
    else TRY(dev_alloc(c, c->Tmp, (size_t)ns * sizeof(double2)));
  }
  if (c->ws_s < s || c->ws_m < m) c->release_workspace();
  TRY(dev_alloc(c, c->V, (size_t)((m + 1) * ns) * sizeof(double2)));
  TRY(dev_alloc(c, c->Z, (size_t)(m * ns) * zsz));
  TRY(dev_alloc(c, c->Bint, (size_t)ns * sizeof(double2)));
  TRY(dev_alloc(c, c->Xint, (size_t)ns * sizeof(double2)));
  // A z_j from the single-precision stencil lands in complex64 (its values
  // are FP32 ones); Gram-Schmidt widens it and writes v_{j+1} in complex128
  if (kprec == ORAS_C64) TRY(dev_alloc(c, c->W32, (size_t)ns * sizeof(float2)));
  TRY(dev_alloc(c, c->partial, (size_t)nblk * (m + 1) * s * sizeof(double2)));
  // small per-column state
  const size_t sH = (size_t)(m + 1) * m * s, sG = (size_t)(m + 1) * s;
  const size_t small_bytes = sizeof(double2) * (sH + sG * 4 + (size_t)m * s) + sizeof(double) * (sG + (size_t)m * s + 8 * s) +
                             sizeof(int) * 8 * s + 4096;
  TRY(dev_alloc(c, c->small, small_bytes));
  c->ws_s = std::max(c->ws_s, s);
  c->ws_m = std::max(c->ws_m, m);
  TRY(ensure_oras_ws(c, s));
  char* sp = c->small.as<char>();
  auto carve = [&](size_t bytes) { char* p = sp; sp += (bytes + 255) / 256 * 256; return (void*)p; };
  double2* H = (double2*)carve(sizeof(double2) * sH);
  double2* g = (double2*)carve(sizeof(double2) * sG);
  double2* hv = (double2*)carve(sizeof(double2) * sG);
  double2* hs = (double2*)carve(sizeof(double2) * sG);
  double2* y = (double2*)carve(sizeof(double2) * sG);
  double2* sn = (double2*)carve(sizeof(double2) * (size_t)m * s);
  double* scale = (double*)carve(sizeof(double) * sG);
  double* cs = (double*)carve(sizeof(double) * (size_t)m * s);
  double* bnorm = (double*)carve(sizeof(double) * s);
  double* beta = (double*)carve(sizeof(double) * s);
  double* est = (double*)carve(sizeof(double) * s);
  double* hnorm = (double*)carve(sizeof(double) * s);
  int* jc = (int*)carve(sizeof(int) * s);
  int* done = (int*)carve(sizeof(int) * s);
  int* conv_d = (int*)carve(sizeof(int) * s);
  double* npart = (double*)c->partial.p;
  double2* dpart = (double2*)c->partial.p;

  double2* V = c->V.as<double2>();
  double2* B = c->Bint.as<double2>();
  double2* X = c->Xint.as<double2>();
  const int conj = (o.flags & ORAS_CONJ) ? 1 : 0;
  launch_to_internal((const double2*)b_dev, B, n, nrhs, (int)s, conj, st);
  if (o.flags & ORAS_X0) launch_to_internal((const double2*)x_dev, X, n, nrhs, (int)s, conj, st);
  else launch_zero(X, (size_t)ns * sizeof(double2), st);
  launch_colnorm2(B, n, (int)s, npart, nblk, st);
  launch_finish_norm(npart, nblk, (int)s, bnorm, st);
  std::vector<double> h_bnorm(s), h_beta(s);
  std::vector<int> h_conv(s, 0), h_done(s, 0), h_iters(s, 0);
  HIP_TRY(c, hipMemcpyAsync(h_bnorm.data(), bnorm, s * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(c, hipGetLastError());

  hipEvent_t ev[4];
  for (int i = 0; i < 4; ++i) HIP_TRY(c, hipEventCreate(&ev[i]));
  double t_sten = 0, t_oras = 0, t_orth = 0;
  int cycles = 0, total = 0;
  oras_status result = ORAS_OK;

  auto true_residual = [&]() -> oras_status {
    TRY(stencil_internal(c, X, B, V, (int)s, ORAS_C128));
    launch_colnorm2(V, n, (int)s, npart, nblk, st);
    launch_finish_norm(npart, nblk, (int)s, beta, st);
    HIP_TRY(c, hipMemcpyAsync(h_beta.data(), beta, s * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipStreamSynchronize(st));
    for (long long col = 0; col < s; ++col) {
      if (!std::isfinite(h_beta[col])) return fail(c, ORAS_E_NUMERIC, "non-finite residual");
      h_conv[col] = (h_bnorm[col] == 0.0) || (h_beta[col] <= tol * h_bnorm[col]);
    }
    return ORAS_OK;
  };

  oras_status rs = true_residual();
  if (rs != ORAS_OK) result = rs;
  while (result == ORAS_OK) {
    bool any = false;
    for (long long col = 0; col < s; ++col) any |= !h_conv[col];
    if (!any || total >= o.maxit) break;
    HIP_TRY(c, hipMemcpyAsync(conv_d, h_conv.data(), s * sizeof(int), hipMemcpyHostToDevice, st));
    launch_cycle_init((int)s, m, beta, conv_d, g, scale, jc, done, st);
    for (long long col = 0; col < s; ++col) h_done[col] = h_conv[col];
    int j = 0;
    for (; j < m; ++j) {
      void* Zj = c->Z.as<char>() + (size_t)j * ns * zsz;
      double2* Vj = V + (size_t)j * ns;
      double2* Vn = V + (size_t)(j + 1) * ns;
      HIP_TRY(c, hipEventRecord(ev[0], st));
      TRY(oras_apply_internal(c, Vj, scale + j * s, Zj, (int)s, !z64, nrhs));
      HIP_TRY(c, hipEventRecord(ev[1], st));
      if (kprec == ORAS_C64) {
        const float2* zin = (const float2*)Zj;
        if (convert) {
          launch_cast<float>((const double2*)Zj, c->Tmp64.as<float2>(), ns, st);
          zin = c->Tmp64.as<float2>();
        }
        apply_stencil<float, float2>(c, zin, nullptr, c->W32.as<float2>(), (int)s, st);
      } else {
        const double2* zin = (const double2*)Zj;
        if (convert) {
          launch_widen((const float2*)Zj, c->Tmp.as<double2>(), ns, st);
          zin = c->Tmp.as<double2>();
        }
        apply_stencil<double>(c, zin, nullptr, Vn, (int)s, st);
      }
      HIP_TRY(c, hipEventRecord(ev[2], st));
      if (kprec == ORAS_C64) {
        const float2* w32 = c->W32.as<float2>();
        launch_cgs_dot(V, ns, j + 1, w32, n, (int)s, dpart, nblk, st);
        launch_cgs_finish_dot(dpart, nblk, j + 1, (int)s, scale, hv, hs, st);
        launch_cgs_update(V, ns, j + 1, hs, w32, Vn, n, (int)s, npart, nblk, st);
      } else {
        launch_cgs_dot(V, ns, j + 1, (const double2*)Vn, n, (int)s, dpart, nblk, st);
        launch_cgs_finish_dot(dpart, nblk, j + 1, (int)s, scale, hv, hs, st);
        launch_cgs_update(V, ns, j + 1, hs, (const double2*)Vn, Vn, n, (int)s, npart, nblk, st);
      }
      launch_finish_norm(npart, nblk, (int)s, hnorm, st);
      launch_arnoldi_step(j, m, (int)s, hnorm, hv, H, cs, sn, g, scale + (j + 1) * s, jc, done,
                          bnorm, tol, est, st);
      HIP_TRY(c, hipEventRecord(ev[3], st));
      HIP_TRY(c, hipGetLastError());
      for (long long col = 0; col < s; ++col)
        if (!h_done[col]) h_iters[col] += 1;
      HIP_TRY(c, hipMemcpyAsync(h_done.data(), done, s * sizeof(int), hipMemcpyDeviceToHost, st));
      HIP_TRY(c, hipStreamSynchronize(st));
      float ms = 0;
      HIP_TRY(c, hipEventElapsedTime(&ms, ev[0], ev[1])); t_oras += ms * 1e-3;
      HIP_TRY(c, hipEventElapsedTime(&ms, ev[1], ev[2])); t_sten += ms * 1e-3;
      HIP_TRY(c, hipEventElapsedTime(&ms, ev[2], ev[3])); t_orth += ms * 1e-3;
      ++total;
      bool all = true, bad = false;
      for (long long col = 0; col < s; ++col) {
        all &= (h_done[col] != 0);
        bad |= (h_done[col] == 2);
      }
      if (bad) { result = fail(c, ORAS_E_NUMERIC, "non-finite value in the Arnoldi process"); break; }
      if (all || total >= o.maxit) { ++j; break; }
    }
    if (result != ORAS_OK) break;
    launch_backsolve(m, (int)s, H, g, jc, y, st);
    if (z64)
      launch_update_x<float2>(c->Z.as<float2>(), ns, y, jc, X, n, (int)s, st);
    else
      launch_update_x<double2>(c->Z.as<double2>(), ns, y, jc, X, n, (int)s, st);
    HIP_TRY(c, hipGetLastError());
    ++cycles;
    rs = true_residual();
    if (rs != ORAS_OK) { result = rs; break; }
  }
  for (int i = 0; i < 4; ++i) (void)hipEventDestroy(ev[i]);
  if (result != ORAS_OK) return result;
  // columns with b = 0 return exactly 0
  for (long long col = 0; col < nrhs; ++col)
    if (h_bnorm[col] == 0.0) launch_zero_column(X, n, (int)s, (int)col, st);
  launch_from_internal(X, (double2*)x_dev, n, nrhs, (int)s, conj, st);
  HIP_TRY(c, hipGetLastError());
  HIP_TRY(c, hipStreamSynchronize(st));
  bool allconv = true;
  for (int col = 0; col < nrhs; ++col) allconv &= (h_conv[col] != 0);
  if (info) {
    for (int col = 0; col < nrhs; ++col) {
      if (info->iters) info->iters[col] = h_iters[col];
      if (info->rel_res) info->rel_res[col] = h_bnorm[col] > 0 ? h_beta[col] / h_bnorm[col] : 0.0;
      if (info->converged) info->converged[col] = h_conv[col];
    }
    info->t_solve = now() - t0;
    info->t_stencil = t_sten;
    info->t_oras = t_oras;
    info->t_ortho = t_orth;
    info->cycles = cycles;
    info->total_iters = total;
  }
  if (!allconv) {
    c->err = "some columns did not reach tol within maxit";
    return ORAS_W_NOT_CONVERGED;
  }
  return ORAS_OK;
}

oras_status oras_point_sources(oras_ctx c, const int* idx_host, const double* amp_host, int nrhs,
                               void* b_dev) {
  if (!c) return ORAS_E_ARG;
  if (!idx_host || !b_dev) return fail(c, ORAS_E_ARG, "null indices or output");
  if (nrhs < 1 || nrhs > 4096) return fail(c, ORAS_E_ARG, "nrhs must be 1..4096");
  if (!c->assembled) return fail(c, ORAS_E_STATE, "point_sources before assemble");
  for (int q = 0; q < nrhs; ++q) {
    const int i = idx_host[3 * q], j = idx_host[3 * q + 1], k = idx_host[3 * q + 2];
    if (i < 0 || i >= c->nx || j < 0 || j >= c->ny || k < 0 || k >= c->nz)
      return fail(c, ORAS_E_ARG, "source index outside the grid");
  }
  TRY(check_device(c));
  DevBuf idx, amp;
  TRY(dev_alloc(c, idx, sizeof(int) * 3 * nrhs));
  if (amp_host) TRY(dev_alloc(c, amp, sizeof(double) * 2 * nrhs));
  HIP_TRY(c, hipMemcpyAsync(idx.p, idx_host, sizeof(int) * 3 * nrhs, hipMemcpyHostToDevice, c->stream));
  if (amp_host)
    HIP_TRY(c, hipMemcpyAsync(amp.p, amp_host, sizeof(double) * 2 * nrhs, hipMemcpyHostToDevice,
                              c->stream));
  launch_zero(b_dev, (size_t)c->n * nrhs * sizeof(double2), c->stream);
  launch_point_sources(idx.as<int>(), amp_host ? amp.as<double>() : nullptr, nrhs,
                       c->px.as<double2>(), c->py.as<double2>(), c->pz.as<double2>(), c->nx, c->ny,
                       c->nz, (double2*)b_dev, c->stream);
  HIP_TRY(c, hipGetLastError());
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  idx.release();
  amp.release();
  return ORAS_OK;
}

oras_status oras_sample(oras_ctx c, const void* u_dev, int nrhs, const int* rec_dev, int nrec,
                        void* d_dev) {
  if (!c) return ORAS_E_ARG;
  if (!u_dev || !rec_dev || !d_dev) return fail(c, ORAS_E_ARG, "null pointer");
  if (nrhs < 1 || nrec < 1) return fail(c, ORAS_E_ARG, "nrhs and nrec must be >= 1");
  if (!c->assembled) return fail(c, ORAS_E_STATE, "sample before assemble");
  TRY(check_device(c));
  TRY(check_receivers(c, rec_dev, nrec));
  launch_sample((const double2*)u_dev, c->n, nrhs, rec_dev, nrec, c->nx, c->ny, (double2*)d_dev,
                c->stream);
  HIP_TRY(c, hipGetLastError());
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return ORAS_OK;
}

oras_status oras_spread(oras_ctx c, const void* d_dev, int nrhs, const int* rec_dev, int nrec,
                        void* b_dev) {
  if (!c) return ORAS_E_ARG;
  if (!d_dev || !rec_dev || !b_dev) return fail(c, ORAS_E_ARG, "null pointer");
  if (nrhs < 1 || nrec < 1) return fail(c, ORAS_E_ARG, "nrhs and nrec must be >= 1");
  if (!c->assembled) return fail(c, ORAS_E_STATE, "spread before assemble");
  TRY(check_device(c));
  TRY(check_receivers(c, rec_dev, nrec));
  launch_zero(b_dev, (size_t)c->n * nrhs * sizeof(double2), c->stream);
  launch_spread((const double2*)d_dev, c->n, nrhs, rec_dev, nrec, c->nx, c->ny, (double2*)b_dev,
                c->stream);
  HIP_TRY(c, hipGetLastError());
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return ORAS_OK;
}

oras_status oras_gradient(oras_ctx c, const void* u_dev, const void* mu_dev, int nrhs,
                          double* g_dev) {
  return oras_gradient_ex(c, u_dev, mu_dev, nrhs, 0, g_dev);
}

oras_status oras_gradient_ex(oras_ctx c, const void* u_dev, const void* mu_dev, int nrhs,
                             int flags, double* g_dev) {
  if (!c) return ORAS_E_ARG;
  if (!u_dev || !mu_dev || !g_dev) return fail(c, ORAS_E_ARG, "null pointer");
  if (nrhs < 1) return fail(c, ORAS_E_ARG, "nrhs must be >= 1");
  if (flags & ~ORAS_GRAD_WEIGHTS) return fail(c, ORAS_E_ARG, "unknown gradient flags");
  if (!c->assembled) return fail(c, ORAS_E_STATE, "gradient before assemble");
  const bool weights = (flags & ORAS_GRAD_WEIGHTS) != 0;
  if (weights && !c->weights_match_m)
    return fail(c, ORAS_E_STATE,
                "weight gradient needs weights that follow m (frozen by the last set_m)");
  TRY(check_device(c));
  launch_gradient(opview(c), c->qf.as<double2>(), (const double2*)u_dev, (const double2*)mu_dev,
                  nrhs, g_dev, c->stream);
  if (weights) {
    const long long sc = weight_grad_scratch(c->nx, c->ny, c->nz);
    TRY(check_free(c, (double)sc * sizeof(double) - (double)c->gradw.bytes));
    TRY(dev_alloc(c, c->gradw, (size_t)sc * sizeof(double)));
    const Table& t = weight_table();
    launch_weight_gradient(opview(c), c->qf.as<double2>(), c->wtab.as<double>(), t.count, t.g0,
                           t.dg, (const double2*)u_dev, (const double2*)mu_dev, nrhs,
                           c->gradw.as<double>(), g_dev, c->stream);
  }
  HIP_TRY(c, hipGetLastError());
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return ORAS_OK;
}

}  // extern "C"
