// Operator assembly on the device: node fields, PML profiles and the 27
// coefficients of every row of A (global grid) or of B_j (one subdomain box).
//
// Paper eq. (1) (Helmholtz equation, k = omega / c, complex c in viscous
// media) discretised by the compact 27-point lambda-adaptive stencil
// (sec. 2.3, FDFD): stiffness mixed over three rotated systems, consistent
// mass, weights looked up per node from a table indexed by G = lambda / h.
// The local matrices B_j of ORAS (sec. 2.1) cut every flux across an
// interior interface and add a Robin (impedance) term on the interface.
//
// Each row is built from its staggered points.  A stiffness family with
// gradient axes `mask` places points at i + sigma/2 (sigma_a = +-1 on the
// mask axes); the gradient along axis a at that point averages the
// differences over the point's 2^(dim-1) edges parallel to a, so the
// coupling of row i to a support node j of the point is
//     -W_a * s_a(j) / 4^(dim-1),   s_a(j) = +1 if j is on i's side along a,
//                                             -1 otherwise,
// summed over the point's axes, with W_a = f * wbar * K_a / h^2, wbar the
// mean family weight of the support nodes, K_a = S / s_a^2 the PML metric at
// the point and f = 1/2 for the in-plane family (each axis lies in two
// planes), 1 otherwise.
#include <algorithm>
#include <cfloat>

#include "oras_internal.h"

namespace oras {

namespace {

__device__ inline double2 csqrt(double2 z) {
  double r = hypot(z.x, z.y);
  if (r == 0.0) return make_double2(0.0, 0.0);
  double t = sqrt(0.5 * (r + fabs(z.x)));
  if (z.x >= 0.0) return make_double2(t, z.y / (2.0 * t));
  return make_double2(fabs(z.y) / (2.0 * t), copysign(t, z.y));
}

__device__ inline bool in_grid(const int p[3], const int n[3]) {
  return p[0] >= 0 && p[0] < n[0] && p[1] >= 0 && p[1] < n[1] && p[2] >= 0 && p[2] < n[2];
}
__device__ inline bool in_box(const int p[3], const int lo[3], const int hi[3]) {
  return p[0] >= lo[0] && p[0] < hi[0] && p[1] >= lo[1] && p[1] < hi[1] && p[2] >= lo[2] &&
         p[2] < hi[2];
}
__device__ inline long long clamp_index(const int p[3], const int n[3]) {
  int x = min(max(p[0], 0), n[0] - 1);
  int y = min(max(p[1], 0), n[1] - 1);
  int z = min(max(p[2], 0), n[2] - 1);
  return ((long long)z * n[1] + y) * n[0] + x;
}
// Interface PML of one subdomain (PML transmission conditions, sec. 2.2 note
// on the size of overlap): extra absorption over the overlap layers beyond the
// owned range on each interior side, sigma = smax (d / L)^power with d the
// distance from the owned range.  smax = 0 on sides without a layer.
struct SubPml {
  int olo[3], ohi[3];
  double smax_lo[3], smax_hi[3], L_lo[3], L_hi[3];
  double h, inv_omega;
  int power;
};

// Stretching factor s_a at half-grid index t (xi = (t - 1) / 2): the outer PML
// profile, plus the subdomain's interface layer when sp is given.
__device__ inline double2 prof_at(const OpView& V, int a, int t, const SubPml* sp = nullptr) {
  double2 s = a == 0 ? V.px[t] : (a == 1 ? V.py[t] : V.pz[t]);
  if (sp) {
    const double xi = 0.5 * (t - 1);
    double sig = 0.0;
    const double d[2] = {sp->h * fmax(0.0, sp->olo[a] - xi), sp->h * fmax(0.0, xi - (sp->ohi[a] - 1))};
    const double L[2] = {sp->L_lo[a], sp->L_hi[a]};
    const double sm[2] = {sp->smax_lo[a], sp->smax_hi[a]};
    for (int side = 0; side < 2; ++side) {
      if (sm[side] <= 0.0) continue;
      const double r = d[side] / L[side];
      double f = 1.0;
      for (int q = 0; q < sp->power; ++q) f *= r;
      sig += sm[side] * f;
    }
    s.y += sig * sp->inv_omega;
  }
  return s;
}
__device__ inline double2 node_S(const OpView& V, const int p[3], const SubPml* sp = nullptr) {
  return cmul(cmul(prof_at(V, 0, 2 * p[0] + 1, sp), prof_at(V, 1, 2 * p[1] + 1, sp)),
              prof_at(V, 2, 2 * p[2] + 1, sp));
}

// The 27 coefficients of the row of node `pos`.  restrict = true builds B_j
// for the box [lo, hi) with Robin interfaces (cut fluxes, impedance term);
// otherwise the row of A, assembled with the interface PML `sp` when given
// (the caller then drops the couplings that leave the box).
__device__ void row_coeffs(const OpView& V, const int pos[3], const int lo[3], const int hi[3],
                           bool restrict_, double2 out[27], const SubPml* sp = nullptr) {
  const int n[3] = {V.nx, V.ny, V.nz};
  for (int e = 0; e < 27; ++e) out[e] = make_double2(0.0, 0.0);
  const double inv_h2 = 1.0 / (V.h * V.h);

  // stiffness: 7 classes of staggered points
  const int masks[7] = {1, 2, 4, 3, 5, 6, 7};
  for (int cls = 0; cls < 7; ++cls) {
    const int mask = masks[cls];
    const int dim = __popc(mask);
    const int widx = dim - 1;                 // w1, w2, w3
    const double ffac = (dim == 2) ? 0.5 : 1.0;
    const double dscale = (dim == 1) ? 1.0 : (dim == 2 ? 0.25 : 0.0625);
    const int npts = 1 << dim;
    for (int sg = 0; sg < npts; ++sg) {
      int sigma[3] = {0, 0, 0};
      {
        int bit = 0;
        for (int a = 0; a < 3; ++a)
          if (mask & (1 << a)) { sigma[a] = ((sg >> bit) & 1) ? 1 : -1; ++bit; }
      }
      // support nodes: tau_a in {0, sigma_a} on the mask axes
      bool valid = true;
      double wsum = 0.0;
      for (int t = 0; t < npts; ++t) {
        int q[3] = {pos[0], pos[1], pos[2]};
        int bit = 0;
        for (int a = 0; a < 3; ++a)
          if (mask & (1 << a)) { if ((t >> bit) & 1) q[a] += sigma[a]; ++bit; }
        if (restrict_) {
          bool g = in_grid(q, n);
          if (g && !in_box(q, lo, hi)) valid = false;
        }
        wsum += V.w7[clamp_index(q, n) * 7 + widx];
      }
      if (!valid) continue;
      const double wbar = wsum / npts;
      double2 sv[3];
      for (int a = 0; a < 3; ++a) {
        int t = (mask & (1 << a)) ? 2 * pos[a] + sigma[a] + 1 : 2 * pos[a] + 1;
        sv[a] = prof_at(V, a, t, sp);
      }
      const double2 S = cmul(cmul(sv[0], sv[1]), sv[2]);
      double2 W[3];
      for (int a = 0; a < 3; ++a) {
        if (mask & (1 << a)) {
          double2 K = cdiv(S, cmul(sv[a], sv[a]));
          W[a] = cscale(K, ffac * wbar * inv_h2 * dscale);
        } else {
          W[a] = make_double2(0.0, 0.0);
        }
      }
      for (int t = 0; t < npts; ++t) {
        int q[3] = {pos[0], pos[1], pos[2]};
        int tau[3] = {0, 0, 0};
        int bit = 0;
        for (int a = 0; a < 3; ++a)
          if (mask & (1 << a)) { if ((t >> bit) & 1) { tau[a] = sigma[a]; q[a] += sigma[a]; } ++bit; }
        if (!in_grid(q, n)) continue;          // Dirichlet ghost: u = 0
        double2 val = make_double2(0.0, 0.0);
        for (int a = 0; a < 3; ++a) {
          if (!(mask & (1 << a))) continue;
          if (tau[a] == 0) val = cadd(val, W[a]);
          else val = csub(val, W[a]);
        }
        const int e = eidx(tau[0], tau[1], tau[2]);
        out[e] = csub(out[e], val);
      }
    }
  }

  // consistent mass
  const long long ii = ((long long)pos[2] * n[1] + pos[1]) * n[0] + pos[0];
  const double om2 = V.omega * V.omega;
  const double2 mti = V.mt[ii];
  const double2 Si = node_S(V, pos, sp);
  {
    double2 d = cscale(cmul(mti, Si), om2 * V.w7[ii * 7 + 3]);
    out[13] = cadd(out[13], d);
  }
  for (int ez = -1; ez <= 1; ++ez)
    for (int ey = -1; ey <= 1; ++ey)
      for (int ex = -1; ex <= 1; ++ex) {
        if (ex == 0 && ey == 0 && ez == 0) continue;
        int q[3] = {pos[0] + ex, pos[1] + ey, pos[2] + ez};
        if (!in_grid(q, n)) continue;
        if (restrict_ && !in_box(q, lo, hi)) continue;
        const long long jj = ((long long)q[2] * n[1] + q[1]) * n[0] + q[0];
        const int widx = 3 + abs(ex) + abs(ey) + abs(ez);
        const double wm = 0.5 * (V.w7[ii * 7 + widx] + V.w7[jj * 7 + widx]);
        double2 mm = cscale(cadd(mti, V.mt[jj]), 0.5);
        double2 ss = cscale(cadd(Si, node_S(V, q, sp)), 0.5);
        double2 mu = cscale(cmul(mm, ss), wm * om2);
        const int e = eidx(ex, ey, ez);
        out[e] = cadd(out[e], mu);
      }

  // Robin faces of B_j: i k S / (s_a h) for each interior face through the node
  if (restrict_) {
    const double2 kk = cscale(csqrt(mti), V.omega);
    for (int a = 0; a < 3; ++a) {
      int cnt = 0;
      if (lo[a] > 0 && pos[a] == lo[a]) ++cnt;
      if (hi[a] < n[a] && pos[a] == hi[a] - 1) ++cnt;
      if (cnt == 0) continue;
      double2 sa = prof_at(V, a, 2 * pos[a] + 1);
      double2 r = cdiv(cmul(make_double2(-kk.y, kk.x), Si), sa);   // i k S / s_a
      r = cscale(r, cnt / V.h);
      out[13] = cadd(out[13], r);
    }
  }
}

__global__ void assemble_global_kernel(OpView V, double2* coef) {
  const long long n = (long long)V.nx * V.ny * V.nz;
  const long long node = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= n) return;
  int pos[3];
  pos[0] = (int)(node % V.nx);
  pos[1] = (int)((node / V.nx) % V.ny);
  pos[2] = (int)(node / ((long long)V.nx * V.ny));
  const int lo[3] = {0, 0, 0};
  const int hi[3] = {V.nx, V.ny, V.nz};
  double2 c[27];
  row_coeffs(V, pos, lo, hi, false, c);
  for (int e = 0; e < 27; ++e) {
    coef[e * n + node] = c[e];
  }
}

template <typename T>
__global__ void assemble_local_kernel(OpView V, const SubDesc* subs, T* lca, IfaceView ifc) {
  const SubDesc sd = subs[blockIdx.y];
  const long long nbox = (long long)sd.sx * sd.sy * sd.sz;
  const long long loc = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (loc >= nbox) return;
  int pos[3];
  pos[0] = sd.lo[0] + (int)(loc % sd.sx);
  pos[1] = sd.lo[1] + (int)((loc / sd.sx) % sd.sy);
  pos[2] = sd.lo[2] + (int)(loc / ((long long)sd.sx * sd.sy));
  double2 c[27];
  if (ifc.kind == ORAS_IFACE_PML) {
    // B_j = R_j A(s_j) R_j^T: the operator with the subdomain's stretching
    // profile, couplings to nodes outside the box dropped (Dirichlet beyond it)
    const int n[3] = {V.nx, V.ny, V.nz};
    SubPml sp;
    sp.h = V.h;
    sp.inv_omega = 1.0 / V.omega;
    sp.power = ifc.power;
    for (int a = 0; a < 3; ++a) {
      sp.olo[a] = sd.olo[a];
      sp.ohi[a] = sd.ohi[a];
      sp.L_lo[a] = (sd.olo[a] - sd.lo[a]) * V.h;
      sp.L_hi[a] = (sd.hi[a] - sd.ohi[a]) * V.h;
      const double num = (ifc.power + 1) * ifc.c_ref * log(1.0 / ifc.R0) * 0.5;
      sp.smax_lo[a] = (sd.lo[a] > 0 && sp.L_lo[a] > 0) ? num / sp.L_lo[a] : 0.0;
      sp.smax_hi[a] = (sd.hi[a] < n[a] && sp.L_hi[a] > 0) ? num / sp.L_hi[a] : 0.0;
    }
    row_coeffs(V, pos, sd.lo, sd.hi, false, c, &sp);
    for (int e = 0; e < 27; ++e) {
      const int q[3] = {pos[0] + e % 3 - 1, pos[1] + (e / 3) % 3 - 1, pos[2] + e / 9 - 1};
      if (!in_box(q, sd.lo, sd.hi)) c[e] = make_double2(0.0, 0.0);
    }
  } else {
    row_coeffs(V, pos, sd.lo, sd.hi, true, c);
  }
  T* out = lca + sd.lca_off;
  for (int e = 0; e < 27; ++e) {
    T v;
    v.x = c[e].x;
    v.y = c[e].y;
    out[e * nbox + loc] = v;
  }
}

__global__ void fields_kernel(const double* vel, const double* q, const double* m_override,
                              const double* wtab, int tab_count, double g0, double dg, long long n,
                              double h, double omega, double* w7, double2* qfac, double2* mt,
                              int keep_weights) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (!keep_weights) {
    // weights from the velocity, or (no velocity given) from the squared slowness
    const double c = vel ? vel[i] : 1.0 / sqrt(m_override[i]);
    const double G = 2.0 * M_PI * c / (omega * h);
    double t = (G - g0) / dg;
    t = fmin(fmax(t, 0.0), (double)(tab_count - 1));
    int i0 = (int)floor(t);
    if (i0 > tab_count - 2) i0 = tab_count - 2;
    const double f = t - i0;
    for (int k = 0; k < 7; ++k)
      w7[i * 7 + k] = (1.0 - f) * wtab[i0 * 7 + k] + f * wtab[(i0 + 1) * 7 + k];
  }
  double2 qf;
  if (keep_weights || !vel) {   // set_m: the attenuation factor of the assembly stays
    qf = qfac[i];
  } else {
    qf = make_double2(1.0, 0.0);
    if (q) {
      double2 a = make_double2(1.0, 0.5 / q[i]);
      qf = cmul(a, a);
    }
    qfac[i] = qf;
  }
  const double m = m_override ? m_override[i] : 1.0 / (vel[i] * vel[i]);
  mt[i] = cscale(qf, m);
}

__global__ void pml_kernel(double2* prof, int n, int npml, double h, double omega, double c_ref,
                           double R0, int power, int low, int high) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t > 2 * n) return;
  const double xi = 0.5 * (t - 1);
  double d = 0.0;
  if (npml > 0) {
    if (low) d = fmax(d, npml - xi);
    if (high) d = fmax(d, xi - (n - 1 - npml));
    d *= h;
  }
  double sigma = 0.0;
  if (npml > 0 && d > 0.0) {
    const double L = npml * h;
    const double smax = (power + 1) * c_ref * log(1.0 / R0) / (2.0 * L);
    sigma = smax * pow(d / L, (double)power);
  }
  prof[t] = make_double2(1.0, sigma / omega);
}

// Check of a model array in two fixed-order stages: per work-group the
// maximum over the valid entries and the number of invalid ones (not finite,
// or not above zero), then one work-group over the partials.  out[0] = the
// maximum (-inf if no entry is valid), out[1] = the invalid count; the
// partials follow (out[2 ..]).  A NaN fails every comparison, so it is
// counted as invalid rather than dropped by the maximum.
constexpr int CHECK_BLOCKS = 1024;
__global__ void check_partial_kernel(const double* x, long long n, double* part) {
  __shared__ double red[256];
  __shared__ double cnt[256];
  double m = -INFINITY, bad = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double v = x[i];
    if (v > 0.0 && v <= DBL_MAX) m = fmax(m, v);
    else bad += 1.0;
  }
  red[threadIdx.x] = m;
  cnt[threadIdx.x] = bad;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
      cnt[threadIdx.x] += cnt[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = red[0];
    part[2 * blockIdx.x + 1] = cnt[0];
  }
}

__global__ void check_reduce_kernel(const double* part, int np, double* out) {
  __shared__ double red[256];
  __shared__ double cnt[256];
  double m = -INFINITY, bad = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) {
    m = fmax(m, part[2 * i]);
    bad += part[2 * i + 1];
  }
  red[threadIdx.x] = m;
  cnt[threadIdx.x] = bad;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
      cnt[threadIdx.x] += cnt[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = red[0];
    out[1] = cnt[0];
  }
}

}  // namespace

void launch_assemble_global(const OpView& op, double2* coef, hipStream_t s) {
  const long long n = (long long)op.nx * op.ny * op.nz;
  const int bs = 128;
  hipLaunchKernelGGL(assemble_global_kernel, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, s,
                     op, coef);
}

void launch_assemble_local(const OpView& op, const SubDesc* subs_dev, int nsub, long long max_box,
                           void* lca, int prec, const IfaceView& ifc, hipStream_t s) {
  const int bs = 128;
  dim3 grid((unsigned)((max_box + bs - 1) / bs), (unsigned)nsub);
  if (prec == ORAS_C64)
    hipLaunchKernelGGL(assemble_local_kernel<float2>, grid, dim3(bs), 0, s, op, subs_dev,
                       (float2*)lca, ifc);
  else
    hipLaunchKernelGGL(assemble_local_kernel<double2>, grid, dim3(bs), 0, s, op, subs_dev,
                       (double2*)lca, ifc);
}

void launch_fields(const double* vel, const double* q, const double* m_override, const double* wtab,
                   int tab_count, double g0, double dg, int nx, int ny, int nz, double h,
                   double omega, double* w7, double2* qfac, double2* mt, hipStream_t s,
                   int keep_weights) {
  const long long n = (long long)nx * ny * nz;
  const int bs = 256;
  hipLaunchKernelGGL(fields_kernel, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, s, vel, q,
                     m_override, wtab, tab_count, g0, dg, n, h, omega, w7, qfac, mt, keep_weights);
}

void launch_pml(double2* prof, int n, int npml, double h, double omega, double c_ref, double R0,
                int power, int low, int high, hipStream_t s) {
  const int bs = 256;
  hipLaunchKernelGGL(pml_kernel, dim3((2 * n + 1 + bs - 1) / bs), dim3(bs), 0, s, prof, n, npml,
                     h, omega, c_ref, R0, power, low, high);
}

long long field_check_doubles() { return 2 + 2 * CHECK_BLOCKS; }

void launch_field_check(const double* x, long long n, double* out, hipStream_t s) {
  const int nb = (int)std::min<long long>(CHECK_BLOCKS, std::max<long long>(1, (n + 255) / 256));
  hipLaunchKernelGGL(check_partial_kernel, dim3(nb), dim3(256), 0, s, x, n, out + 2);
  hipLaunchKernelGGL(check_reduce_kernel, dim3(1), dim3(256), 0, s, out + 2, nb, out);
}

}  // namespace oras
