// Stencil-weight part of the misfit gradient when the lambda-adaptive weights
// follow the model (paper sec. 2.3: each node's weights are picked from its
// local G = lambda / h, so they move with the squared slowness m).
//
// g_i -= Re sum_k H_k,i dw_k/dm_i, with H_k,i = sum_s d(mu_s^H A u_s)/dw_k,i
// and dw_k/dm_i = (table slope at G_i) dG/dm_i, dG/dm = -G / (2 m).
//
// Stiffness weights (k = 0, 1, 2: families F1, F2, F3) enter A through the
// family weight of a staggered point, the mean of its support nodes' weights
// (a support node outside the grid takes the weights of the node it clamps
// to).  A staggered point p contributes
//     T_p = -sum_a ffac Scen / (s_a^2 h^2) sum_s conj(D_a mu_s) D_a u_s
// (D_a: the family's averaged difference along axis a over the support,
// fields zero outside the grid), shared by its support nodes as T_p / npts.
// The first kernel forms Re T_p for every staggered point of a family, the
// second gathers them per node (with the clamp multiplicity), adds the mass
// weights' terms (diagonal and shell couplings) and contracts with dw/dm.
#include "oras_internal.h"

namespace oras {

namespace {

__constant__ int kFamMask[7] = {1, 2, 4, 3, 5, 6, 7};

struct FamLayout {
  long long off[7];      // start of each family's array
  int ext[7][3];         // staggered-point extents: n_a + 1 on the family's axes, n_a otherwise
};

__device__ inline double2 prof(const OpView& V, int a, int t) {
  return a == 0 ? V.px[t] : (a == 1 ? V.py[t] : V.pz[t]);
}

// Re T_p for every staggered point of family `fam` (base node b: b_a from -1
// on the family's axes).
__global__ void stagger_sens_kernel(OpView V, FamLayout L, int fam, const double2* __restrict__ u,
                                    const double2* __restrict__ mu, int nrhs,
                                    double* __restrict__ out) {
  const int mask = kFamMask[fam];
  const int dim = __popc(mask);
  const int ex = L.ext[fam][0], ey = L.ext[fam][1], ez = L.ext[fam][2];
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= (long long)ex * ey * ez) return;
  const int idx[3] = {(int)(p % ex), (int)((p / ex) % ey), (int)(p / ((long long)ex * ey))};
  const int n[3] = {V.nx, V.ny, V.nz};
  int b[3];
  double2 s[3];
  for (int a = 0; a < 3; ++a) {
    const bool on = mask & (1 << a);
    b[a] = on ? idx[a] - 1 : idx[a];
    s[a] = prof(V, a, on ? 2 * b[a] + 2 : 2 * b[a] + 1);
  }
  const double2 Scen = cmul(cmul(s[0], s[1]), s[2]);
  const double ffac = dim == 2 ? 0.5 : 1.0;
  const double dscale = dim == 1 ? 1.0 : (dim == 2 ? 0.5 : 0.25);
  const double inv_h2 = 1.0 / (V.h * V.h);
  double2 coef[3];
  for (int a = 0; a < 3; ++a) {
    coef[a] = make_double2(0.0, 0.0);
    if (mask & (1 << a)) {
      // -ffac Scen / (s_a^2 h^2)
      coef[a] = cscale(cdiv(Scen, cmul(s[a], s[a])), -ffac * inv_h2);
    }
  }
  const long long nn = (long long)n[0] * n[1] * n[2];
  const int npts = 1 << dim;
  double acc = 0.0;
  for (int c = 0; c < nrhs; ++c) {
    double2 Dm[3], Du[3];
    for (int a = 0; a < 3; ++a) {
      Dm[a] = make_double2(0.0, 0.0);
      Du[a] = make_double2(0.0, 0.0);
    }
    for (int r = 0; r < npts; ++r) {
      int q[3] = {b[0], b[1], b[2]};
      int sign[3] = {0, 0, 0};
      int bit = 0;
      for (int a = 0; a < 3; ++a)
        if (mask & (1 << a)) {
          const int rho = (r >> bit) & 1;
          q[a] += rho;
          sign[a] = rho ? 1 : -1;
          ++bit;
        }
      if (q[0] < 0 || q[0] >= n[0] || q[1] < 0 || q[1] >= n[1] || q[2] < 0 || q[2] >= n[2])
        continue;                                     // ghost: u = mu = 0
      const long long node = ((long long)q[2] * n[1] + q[1]) * n[0] + q[0];
      const double2 mv = mu[(long long)c * nn + node], uv = u[(long long)c * nn + node];
      for (int a = 0; a < 3; ++a)
        if (mask & (1 << a)) {
          const double d = sign[a] * dscale;
          Dm[a] = cadd(Dm[a], cscale(mv, d));
          Du[a] = cadd(Du[a], cscale(uv, d));
        }
    }
    for (int a = 0; a < 3; ++a)
      if (mask & (1 << a)) {
        double2 t = make_double2(0.0, 0.0);
        cfmaconj(t, Dm[a], Du[a]);                    // conj(D mu) D u
        acc += cmul(coef[a], t).x;
      }
  }
  out[L.off[fam] + p] = acc;
}

// g_i -= sum_k dw_k/dm_i Re H_k,i.
__global__ void weight_grad_kernel(OpView V, FamLayout L, const double* __restrict__ stag,
                                   const double2* __restrict__ qfac, const double* __restrict__ wtab,
                                   int tab_count, double g0, double dg,
                                   const double2* __restrict__ u, const double2* __restrict__ mu,
                                   int nrhs, double* __restrict__ g) {
  const int n[3] = {V.nx, V.ny, V.nz};
  const long long nn = (long long)n[0] * n[1] * n[2];
  const long long node = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= nn) return;
  const int i[3] = {(int)(node % n[0]), (int)((node / n[0]) % n[1]),
                    (int)(node / ((long long)n[0] * n[1]))};
  double H[7] = {0, 0, 0, 0, 0, 0, 0};
  // stiffness weights: staggered points whose (clamped) support holds node i
  for (int fam = 0; fam < 7; ++fam) {
    const int mask = kFamMask[fam];
    const int dim = __popc(mask);
    const double inv_npts = 1.0 / (1 << dim);
    for (int r = 0; r < (1 << dim); ++r) {
      int idx[3];
      int count = 1;
      int bit = 0;
      for (int a = 0; a < 3; ++a) {
        if (mask & (1 << a)) {
          const int ba = i[a] - 1 + ((r >> bit) & 1);     // base i_a - 1 or i_a
          ++bit;
          // support offsets 0, 1 whose clamped node is i_a
          const int c0 = min(max(ba, 0), n[a] - 1) == i[a];
          const int c1 = min(max(ba + 1, 0), n[a] - 1) == i[a];
          count *= c0 + c1;
          idx[a] = ba + 1;
        } else {
          idx[a] = i[a];
        }
      }
      if (count == 0) continue;
      const long long p =
          ((long long)idx[2] * L.ext[fam][1] + idx[1]) * L.ext[fam][0] + idx[0];
      H[dim - 1] += stag[L.off[fam] + p] * count * inv_npts;
    }
  }
  // mass weights: diagonal wm0 and shell couplings
  const double om2 = V.omega * V.omega;
  auto S_at = [&](const int q[3]) {
    return cmul(cmul(V.px[2 * q[0] + 1], V.py[2 * q[1] + 1]), V.pz[2 * q[2] + 1]);
  };
  const double2 Si = S_at(i), mti = V.mt[node];
  {
    double2 t = make_double2(0.0, 0.0);
    for (int c = 0; c < nrhs; ++c) cfmaconj(t, mu[(long long)c * nn + node], u[(long long)c * nn + node]);
    H[3] += om2 * cmul(cmul(mti, Si), t).x;
  }
  for (int ez = -1; ez <= 1; ++ez)
    for (int ey = -1; ey <= 1; ++ey)
      for (int ex = -1; ex <= 1; ++ex) {
        if (ex == 0 && ey == 0 && ez == 0) continue;
        const int q[3] = {i[0] + ex, i[1] + ey, i[2] + ez};
        if (q[0] < 0 || q[0] >= n[0] || q[1] < 0 || q[1] >= n[1] || q[2] < 0 || q[2] >= n[2])
          continue;                                   // ghost: u = mu = 0
        const long long nb = ((long long)q[2] * n[1] + q[1]) * n[0] + q[0];
        const int t = 3 + abs(ex) + abs(ey) + abs(ez);
        const double2 coup = cmul(cscale(cadd(mti, V.mt[nb]), 0.5), cscale(cadd(Si, S_at(q)), 0.5));
        double2 s2 = make_double2(0.0, 0.0);
        for (int c = 0; c < nrhs; ++c) {
          cfmaconj(s2, mu[(long long)c * nn + node], u[(long long)c * nn + nb]);
          cfmaconj(s2, mu[(long long)c * nn + nb], u[(long long)c * nn + node]);
        }
        H[t] += 0.5 * om2 * cmul(coup, s2).x;
      }
  // dw/dm from the piecewise-linear table at G = 2 pi / (omega h sqrt(m))
  const double m = cdiv(mti, qfac[node]).x;
  const double G = 2.0 * M_PI / (V.omega * V.h * sqrt(m));
  const double tt = (G - g0) / dg;
  if (!(tt > 0.0 && tt < tab_count - 1.0)) return;    // clamped: weights do not move
  const int i0 = min((int)floor(tt), tab_count - 2);
  const double dGdm = -G / (2.0 * m);
  double acc = 0.0;
  for (int k = 0; k < 7; ++k) acc += (wtab[(i0 + 1) * 7 + k] - wtab[i0 * 7 + k]) / dg * dGdm * H[k];
  g[node] -= acc;
}

}  // namespace

long long weight_grad_scratch(int nx, int ny, int nz) {
  long long tot = 0;
  const int n[3] = {nx, ny, nz};
  const int masks[7] = {1, 2, 4, 3, 5, 6, 7};
  for (int f = 0; f < 7; ++f) {
    long long e = 1;
    for (int a = 0; a < 3; ++a) e *= (masks[f] & (1 << a)) ? n[a] + 1 : n[a];
    tot += e;
  }
  return tot;
}

void launch_weight_gradient(const OpView& op, const double2* qfac, const double* wtab,
                            int tab_count, double g0, double dg, const double2* u,
                            const double2* mu, int nrhs, double* scratch, double* g,
                            hipStream_t st) {
  FamLayout L;
  const int n[3] = {op.nx, op.ny, op.nz};
  const int masks[7] = {1, 2, 4, 3, 5, 6, 7};
  long long off = 0;
  for (int f = 0; f < 7; ++f) {
    long long e = 1;
    for (int a = 0; a < 3; ++a) {
      L.ext[f][a] = (masks[f] & (1 << a)) ? n[a] + 1 : n[a];
      e *= L.ext[f][a];
    }
    L.off[f] = off;
    off += e;
  }
  const int bs = 128;
  for (int f = 0; f < 7; ++f) {
    const long long e = (long long)L.ext[f][0] * L.ext[f][1] * L.ext[f][2];
    hipLaunchKernelGGL(stagger_sens_kernel, dim3((unsigned)((e + bs - 1) / bs)), dim3(bs), 0, st, op,
                       L, f, u, mu, nrhs, scratch);
  }
  const long long nn = (long long)n[0] * n[1] * n[2];
  hipLaunchKernelGGL(weight_grad_kernel, dim3((unsigned)((nn + bs - 1) / bs)), dim3(bs), 0, st, op,
                     L, scratch, qfac, wtab, tab_count, g0, dg, u, mu, nrhs, g);
}

}  // namespace oras
