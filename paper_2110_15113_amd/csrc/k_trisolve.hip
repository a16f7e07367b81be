// ORAS preconditioner apply on the device:
//     z = M^{-1} v = sum_j R_j^T D_j B_j^{-1} R_j v
// (paper sec. 2.1; sec. 2.2: the local solves act on the whole block of
// right-hand sides at once -- the pseudo-block form).
//
// For every subdomain the local solve runs over the z-planes of its box with
// the plane inverses S_k^{-1} built by the factorisation:
//   forward   t = R_j v |_plane k - L_k y_{k-1};   y_k = S_k^{-1} t
//   backward  t = U_k x_{k+1};                    x_k = y_k - S_k^{-1} t
// and the restricted prolongation writes every node from its owner only
// (Boolean partition of unity), so each output entry is written once and no
// atomics are needed.  All subdomains advance one plane per launch; the
// plane product is a batched complex GEMM (P x P) x (P x s) on MFMA.
//
// Complex products on real MFMA: with A = Ar + i Ai and B = Br + i Bi, the
// interleaved output columns (Re, Im) of C = A B come from two real
// products per k-slice: Ar * [Br | Bi] + Ai * [-Bi | Br].  One 16x16x4
// instruction covers 16 rows x 8 complex columns x 4 complex k.
#include <algorithm>

#include "oras_internal.h"

namespace oras {

namespace {

__device__ inline long long tile_off(int I, int J, int nt) {
  return ((long long)I * nt + J) * (TILE * TILE);
}

// Both 16x16x4 instructions take A[row = lane % 16][k = lane / 16] and
// B[k = lane / 16][col = lane % 16]; the result column is lane % 16, but the
// result row of accumulator item t differs: 4 (lane / 16) + t for FP32,
// lane / 16 + 4 t for FP64 (checked on gfx950).
template <typename R> struct Mfma;
template <> struct Mfma<float> {
  typedef float acc_t __attribute__((ext_vector_type(4)));
  static __device__ inline acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ inline int out_row(int group, int t) { return 4 * group + t; }
};
template <> struct Mfma<double> {
  typedef double acc_t __attribute__((ext_vector_type(4)));
  static __device__ inline acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ inline int out_row(int group, int t) { return group + 4 * t; }
};

// Y_k (=|-=) S_k^{-1} t for one 32-row tile of one subdomain; one wave.
// NS = s / 8 column groups of 8 complex right-hand sides.
template <typename R, int NS>
__global__ void __launch_bounds__(64) plane_gemm_kernel(const SubDesc* subs, int k, int bwd,
                                                        const C<R>* __restrict__ fac,
                                                        C<R>* __restrict__ ybuf,
                                                        const C<R>* __restrict__ tvbuf, int s,
                                                        int c0) {
  using T = C<R>;
  using M = Mfma<R>;
  const SubDesc sd = subs[blockIdx.y];
  if (bwd ? (k > sd.sz - 2) : (k >= sd.sz)) return;
  const int I = blockIdx.x;
  const int nt = sd.nt;
  if (I >= nt) return;
  const int P = sd.P;
  const T* A = fac + sd.fac_off + (long long)k * P * P + tile_off(I, 0, nt);
  const T* Bm = tvbuf + sd.tv_off * (long long)s + c0;
  T* Y = ybuf + (sd.y_off + (long long)k * P) * s + c0;
  const int lane = threadIdx.x;
  const int m = lane & 15, kk = lane >> 4;
  const int bn = m >> 1;
  const bool im = (m & 1) != 0;
  typename M::acc_t acc[2][NS];
#pragma unroll
  for (int rs = 0; rs < 2; ++rs)
#pragma unroll
    for (int ns = 0; ns < NS; ++ns) acc[rs][ns] = typename M::acc_t{0, 0, 0, 0};

  for (int J = 0; J < nt; ++J) {
    const T* tA = A + (long long)J * (TILE * TILE);
#pragma unroll 2
    for (int q = 0; q < 8; ++q) {
      const int kc = J * TILE + q * 4 + kk;
      const T a0 = tA[(q * TILE + m) * 4 + kk];
      const T a1 = tA[(q * TILE + 16 + m) * 4 + kk];
      const T* brow = Bm + (long long)kc * s + bn;
#pragma unroll
      for (int ns = 0; ns < NS; ++ns) {
        const T bv = brow[ns * 8];
        const R b1 = im ? bv.y : bv.x;
        const R b2 = im ? bv.x : -bv.y;
        acc[0][ns] = M::op(a0.x, b1, acc[0][ns]);
        acc[0][ns] = M::op(a0.y, b2, acc[0][ns]);
        acc[1][ns] = M::op(a1.x, b1, acc[1][ns]);
        acc[1][ns] = M::op(a1.y, b2, acc[1][ns]);
      }
    }
  }
#pragma unroll
  for (int rs = 0; rs < 2; ++rs)
#pragma unroll
    for (int ns = 0; ns < NS; ++ns)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = I * TILE + rs * 16 + M::out_row(kk, i);
        R* yr = reinterpret_cast<R*>(Y + (long long)row * s);
        const int idx = ns * 16 + m;
        if (bwd) yr[idx] -= acc[rs][ns][i];
        else yr[idx] = acc[rs][ns][i];
      }
}

// forward right-hand side of plane k: t = (scale * v)|_plane - L_k y_{k-1}
template <typename R>
__global__ void fwd_rhs_kernel(const SubDesc* subs, int k, const C<R>* __restrict__ lca,
                               const C<R>* __restrict__ ybuf, C<R>* __restrict__ tvbuf,
                               const double2* __restrict__ v, const double* __restrict__ scale,
                               int nx, int ny, int s) {
  using T = C<R>;
  const SubDesc sd = subs[blockIdx.y];
  if (k >= sd.sz) return;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)sd.P * s) return;
  const int q = (int)(idx / s), c = (int)(idx % s);
  T t;
  t.x = 0;
  t.y = 0;
  if (q < sd.p) {
    const int qx = q % sd.sx, qy = q / sd.sx;
    const long long g = ((long long)(sd.lo[2] + k) * ny + sd.lo[1] + qy) * nx + sd.lo[0] + qx;
    double2 vv = v[g * s + c];
    const double sc = scale ? scale[c] : 1.0;
    t.x = (R)(vv.x * sc);
    t.y = (R)(vv.y * sc);
    if (k > 0) {
      const long long nbox = (long long)sd.sx * sd.sy * sd.sz;
      const long long node = ((long long)k * sd.sy + qy) * sd.sx + qx;
      const T* L = lca + sd.lca_off;
      const T* Yp = ybuf + (sd.y_off + (long long)(k - 1) * sd.P) * s;
      for (int dy = -1; dy <= 1; ++dy) {
        const int py = qy + dy;
        if (py < 0 || py >= sd.sy) continue;
        for (int dx = -1; dx <= 1; ++dx) {
          const int px = qx + dx;
          if (px < 0 || px >= sd.sx) continue;
          const T l = L[eidx(dx, dy, -1) * nbox + node];
          const T y = Yp[(long long)(py * sd.sx + px) * s + c];
          t.x -= l.x * y.x - l.y * y.y;
          t.y -= l.x * y.y + l.y * y.x;
        }
      }
    }
  }
  tvbuf[sd.tv_off * (long long)s + idx] = t;
}

// backward right-hand side of plane k: t = U_k x_{k+1}
template <typename R>
__global__ void bwd_rhs_kernel(const SubDesc* subs, int k, const C<R>* __restrict__ lca,
                               const C<R>* __restrict__ ybuf, C<R>* __restrict__ tvbuf, int s) {
  using T = C<R>;
  const SubDesc sd = subs[blockIdx.y];
  if (k > sd.sz - 2) return;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)sd.P * s) return;
  const int q = (int)(idx / s), c = (int)(idx % s);
  T t;
  t.x = 0;
  t.y = 0;
  if (q < sd.p) {
    const int qx = q % sd.sx, qy = q / sd.sx;
    const long long nbox = (long long)sd.sx * sd.sy * sd.sz;
    const long long node = ((long long)k * sd.sy + qy) * sd.sx + qx;
    const T* L = lca + sd.lca_off;
    const T* Yn = ybuf + (sd.y_off + (long long)(k + 1) * sd.P) * s;
    for (int dy = -1; dy <= 1; ++dy) {
      const int py = qy + dy;
      if (py < 0 || py >= sd.sy) continue;
      for (int dx = -1; dx <= 1; ++dx) {
        const int px = qx + dx;
        if (px < 0 || px >= sd.sx) continue;
        const T u = L[eidx(dx, dy, 1) * nbox + node];
        const T y = Yn[(long long)(py * sd.sx + px) * s + c];
        t.x += u.x * y.x - u.y * y.y;
        t.y += u.x * y.y + u.y * y.x;
      }
    }
  }
  tvbuf[sd.tv_off * (long long)s + idx] = t;
}

// restricted prolongation: every global node takes its owner's local value
template <typename R, typename Z>
__global__ void prolong_kernel(const SubDesc* subs, const int* __restrict__ owner, int px, int py,
                               const C<R>* __restrict__ ybuf, Z* __restrict__ z, int nx, int ny,
                               int nz, int s) {
  const long long n = (long long)nx * ny * nz;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * s) return;
  const long long node = idx / s;
  const int c = (int)(idx % s);
  const int i = (int)(node % nx);
  const int j = (int)((node / nx) % ny);
  const int kz = (int)(node / ((long long)nx * ny));
  const int sub = owner[i] + px * (owner[nx + j] + py * owner[nx + ny + kz]);
  const SubDesc sd = subs[sub];
  const int lx = i - sd.lo[0], ly = j - sd.lo[1], lz = kz - sd.lo[2];
  const C<R> val = ybuf[(sd.y_off + (long long)lz * sd.P + ly * sd.sx + lx) * s + c];
  Z o;
  o.x = val.x;
  o.y = val.y;
  z[idx] = o;
}

template <typename R, int NS>
void gemm_launch(const SubDesc* subs, int nsub, int k, int bwd, int max_nt, const C<R>* fac,
                 C<R>* ybuf, const C<R>* tvbuf, int s, int c0, hipStream_t st) {
  hipLaunchKernelGGL((plane_gemm_kernel<R, NS>), dim3(max_nt, nsub), dim3(64), 0, st, subs, k, bwd,
                     fac, ybuf, tvbuf, s, c0);
}

// Columns in chunks of at most 64 right-hand sides (8 groups of 8).
template <typename R>
void gemm_dispatch(const SubDesc* subs, int nsub, int k, int bwd, int max_nt, const C<R>* fac,
                   C<R>* ybuf, const C<R>* tvbuf, int s, hipStream_t st) {
  for (int c0 = 0; c0 < s; c0 += 8 * RHS_ALIGN) {
    const int groups = std::min(8, (s - c0) / RHS_ALIGN);
    switch (groups) {
      case 1: gemm_launch<R, 1>(subs, nsub, k, bwd, max_nt, fac, ybuf, tvbuf, s, c0, st); break;
      case 2: gemm_launch<R, 2>(subs, nsub, k, bwd, max_nt, fac, ybuf, tvbuf, s, c0, st); break;
      case 3: gemm_launch<R, 3>(subs, nsub, k, bwd, max_nt, fac, ybuf, tvbuf, s, c0, st); break;
      case 4: gemm_launch<R, 4>(subs, nsub, k, bwd, max_nt, fac, ybuf, tvbuf, s, c0, st); break;
      case 5: gemm_launch<R, 5>(subs, nsub, k, bwd, max_nt, fac, ybuf, tvbuf, s, c0, st); break;
      case 6: gemm_launch<R, 6>(subs, nsub, k, bwd, max_nt, fac, ybuf, tvbuf, s, c0, st); break;
      case 7: gemm_launch<R, 7>(subs, nsub, k, bwd, max_nt, fac, ybuf, tvbuf, s, c0, st); break;
      default: gemm_launch<R, 8>(subs, nsub, k, bwd, max_nt, fac, ybuf, tvbuf, s, c0, st); break;
    }
  }
}

}  // namespace

template <typename R, typename Z>
void launch_oras_apply(const SubDesc* subs_dev, int nsub, int max_sz, int max_nt, long long max_p,
                       const C<R>* fac, const C<R>* lca, C<R>* ybuf, C<R>* tvbuf,
                       const double2* v, const double* scale, Z* z, int nx, int ny, int nz,
                       int s, const int* owner_dev, int parts_x, int parts_y, hipStream_t st,
                       hipEvent_t* gemm_ev) {
  const int bs = 256;
  int step = 0;
  auto mark = [&](int which) {
    if (gemm_ev) (void)hipEventRecord(gemm_ev[2 * step + which], st);
  };
  const dim3 grhs((unsigned)((max_p * s + bs - 1) / bs), (unsigned)nsub);
  for (int k = 0; k < max_sz; ++k) {
    hipLaunchKernelGGL((fwd_rhs_kernel<R>), grhs, dim3(bs), 0, st, subs_dev, k, lca, ybuf, tvbuf,
                       v, scale, nx, ny, s);
    mark(0);
    gemm_dispatch<R>(subs_dev, nsub, k, 0, max_nt, fac, ybuf, tvbuf, s, st);
    mark(1);
    ++step;
  }
  for (int k = max_sz - 2; k >= 0; --k) {
    hipLaunchKernelGGL((bwd_rhs_kernel<R>), grhs, dim3(bs), 0, st, subs_dev, k, lca, ybuf, tvbuf,
                       s);
    mark(0);
    gemm_dispatch<R>(subs_dev, nsub, k, 1, max_nt, fac, ybuf, tvbuf, s, st);
    mark(1);
    ++step;
  }
  // owner map: owner_dev[0..nx) x part, [nx, nx+ny) y part, [nx+ny, ..) z part
  const long long n = (long long)nx * ny * nz;
  hipLaunchKernelGGL((prolong_kernel<R, Z>), dim3((unsigned)((n * s + bs - 1) / bs)), dim3(bs), 0,
                     st, subs_dev, owner_dev, parts_x, parts_y, ybuf, z, nx, ny, nz, s);
}

template void launch_oras_apply<float, float2>(const SubDesc*, int, int, int, long long,
                                               const float2*, const float2*, float2*, float2*,
                                               const double2*, const double*, float2*, int, int,
                                               int, int, const int*, int, int, hipStream_t,
                                               hipEvent_t*);
template void launch_oras_apply<float, double2>(const SubDesc*, int, int, int, long long,
                                                const float2*, const float2*, float2*, float2*,
                                                const double2*, const double*, double2*, int,
                                                int, int, int, const int*, int, int, hipStream_t,
                                               hipEvent_t*);
template void launch_oras_apply<double, double2>(const SubDesc*, int, int, int, long long,
                                                 const double2*, const double2*, double2*,
                                                 double2*, const double2*, const double*,
                                                 double2*, int, int, int, int, const int*, int,
                                                 int, hipStream_t, hipEvent_t*);

}  // namespace oras
