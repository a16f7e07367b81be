// ORAS preconditioner apply on the device:
//     z = M^{-1} v = sum_j R_j^T D_j B_j^{-1} R_j v
// (paper sec. 2.1; sec. 2.2: the local solves act on the whole block of
// right-hand sides at once -- the pseudo-block form).
//
// For every subdomain the local solve runs over the z-planes of its box with
// the plane inverses S_k^{-1} built by the factorisation:
//   forward   t = R_j v |_plane k - L_k y_{k-1};   y_k = S_k^{-1} t
//   backward  t = U_k x_{k+1};                    x_k = y_k - S_k^{-1} t
// All subdomains advance one plane per pair of launches (subdomains are
// independent, so no inter-work-group synchronisation is ever needed):
//   * a right-hand-side kernel forms t for the plane of every subdomain
//     (the restriction from the global vector is fused in);
//   * a GEMM kernel with one wave per (subdomain, 32-row tile) streams its
//     rows of S_k^{-1} from HBM and t from L2 into MFMA.  (Measured on
//     gfx950 against variants staging t through LDS for 1-8 waves and
//     against persistent balanced workers with register prefetch: this
//     simplest form was the fastest.)
// The GEMM epilogue stores the plane's rows and, once a plane is final,
// writes the owned nodes to the output (restricted prolongation with a
// Boolean partition of unity: each output entry is written once, no
// atomics).
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

template <typename Z> struct Comp;
template <> struct Comp<float2> { typedef float type; };
template <> struct Comp<double2> { typedef double type; };

// Plane right-hand sides of all subdomains: forward t = scale * v|_plane -
// L_k y_{k-1}, backward t = U_k x_{k+1}; rows beyond the plane are zero.
template <typename R>
__global__ void plane_rhs_kernel(const SubDesc* __restrict__ subs, int k, int bwd,
                                 const C<R>* __restrict__ lca, const C<R>* __restrict__ ybuf,
                                 C<R>* __restrict__ tvbuf, const double2* __restrict__ v,
                                 const double* __restrict__ scale, int nx, int ny, int s) {
  using T = C<R>;
  const SubDesc sd = subs[blockIdx.y];
  if (bwd ? (k > sd.sz - 2) : (k >= sd.sz)) return;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)sd.P * s) return;
  const int q = (int)(idx / s), c = (int)(idx % s);
  T t;
  t.x = 0;
  t.y = 0;
  if (q < sd.p) {
    const int qx = q % sd.sx, qy = q / sd.sx;
    if (!bwd) {
      const long long g = ((long long)(sd.lo[2] + k) * ny + sd.lo[1] + qy) * nx + sd.lo[0] + qx;
      const double2 vv = v[g * s + c];
      const double sc = scale ? scale[c] : 1.0;
      t.x = (R)(vv.x * sc);
      t.y = (R)(vv.y * sc);
    }
    if (bwd || k > 0) {
      const long long nbox = (long long)sd.sx * sd.sy * sd.sz;
      const long long node = ((long long)k * sd.sy + qy) * sd.sx + qx;
      const T* L = lca + sd.lca_off;
      const T* Yn = ybuf + (sd.y_off + (long long)(bwd ? k + 1 : k - 1) * sd.P) * s;
      const int ez = bwd ? 1 : -1;
      const R sg = bwd ? (R)1 : (R)-1;
      for (int dy = -1; dy <= 1; ++dy) {
        const int py = qy + dy;
        if (py < 0 || py >= sd.sy) continue;
        for (int dx = -1; dx <= 1; ++dx) {
          const int px = qx + dx;
          if (px < 0 || px >= sd.sx) continue;
          const T l = L[eidx(dx, dy, ez) * nbox + node];
          const T y = Yn[(long long)(py * sd.sx + px) * s + c];
          t.x += sg * (l.x * y.x - l.y * y.y);
          t.y += sg * (l.x * y.y + l.y * y.x);
        }
      }
    }
  }
  tvbuf[sd.tv_off * (long long)s + idx] = t;
}

// Y_k (=|-=) S_k^{-1} t for one 32-row tile of one subdomain: one wave,
// S_k^{-1} rows streamed from HBM (one contiguous 8 KB tile per k-chunk),
// t read through L1/L2 (it is shared by the subdomain's row tiles).  A
// 16-row x 8-column x 4-k step is two MFMAs (real and imaginary part of A).
template <typename R, typename Z, int NS>
__global__ void __launch_bounds__(64)
plane_gemm_kernel(const SubDesc* __restrict__ subs, int k, int bwd, const C<R>* __restrict__ fac,
                   const C<R>* __restrict__ tvbuf, C<R>* __restrict__ ybuf, Z* __restrict__ z,
                   int nx, int ny, int s, int c0) {
  using T = C<R>;
  using M = Mfma<R>;
  using ZR = typename Comp<Z>::type;
  const SubDesc sd = subs[blockIdx.y];
  if (bwd ? (k > sd.sz - 2) : (k >= sd.sz)) return;
  const int I = blockIdx.x;
  const int nt = sd.nt;
  if (I >= nt) return;
  const int P = sd.P;
  const T* A = fac + sd.fac_off + (long long)k * P * P + tile_off(I, 0, nt);
  const T* Bm = tvbuf + sd.tv_off * (long long)s + c0;
  T* Yk = ybuf + (sd.y_off + (long long)k * P) * s;
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
  const bool final_plane = bwd || (k == sd.sz - 1);
#pragma unroll
  for (int rs = 0; rs < 2; ++rs)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = I * TILE + rs * 16 + M::out_row(kk, i);
      R* yr = reinterpret_cast<R*>(Yk + (long long)row * s + c0);
      long long zoff = -1;
      if (final_plane && row < sd.p) {
        const int qx = row % sd.sx, qy = row / sd.sx;
        const int gx = sd.lo[0] + qx, gy = sd.lo[1] + qy, gz = sd.lo[2] + k;
        if (gx >= sd.olo[0] && gx < sd.ohi[0] && gy >= sd.olo[1] && gy < sd.ohi[1] &&
            gz >= sd.olo[2] && gz < sd.ohi[2])
          zoff = (((long long)gz * ny + gy) * nx + gx) * s + c0;
      }
#pragma unroll
      for (int ns = 0; ns < NS; ++ns) {
        const int idx = ns * 16 + m;
        R val = acc[rs][ns][i];
        if (bwd) val = yr[idx] - val;
        yr[idx] = val;
        if (zoff >= 0) reinterpret_cast<ZR*>(z + zoff)[idx] = (ZR)val;
      }
    }
}

template <typename R, typename Z, int NS>
void gemm_launch(const SubDesc* subs, int nsub, int max_nt, int k, int bwd, const C<R>* fac,
                 const C<R>* tvbuf, C<R>* ybuf, Z* z, int nx, int ny, int s, int c0,
                 hipStream_t st) {
  hipLaunchKernelGGL((plane_gemm_kernel<R, Z, NS>), dim3(max_nt, nsub), dim3(64), 0, st, subs, k,
                     bwd, fac, tvbuf, ybuf, z, nx, ny, s, c0);
}

// Columns in chunks of at most 64 right-hand sides (8 groups of 8).
template <typename R, typename Z>
void gemm_dispatch(const SubDesc* subs, int nsub, int max_nt, int k, int bwd, const C<R>* fac,
                   const C<R>* tvbuf, C<R>* ybuf, Z* z, int nx, int ny, int s, hipStream_t st) {
  for (int c0 = 0; c0 < s; c0 += 8 * RHS_ALIGN) {
    const int groups = std::min(8, (s - c0) / RHS_ALIGN);
#define ORAS_GEMM(NS_) \
  gemm_launch<R, Z, NS_>(subs, nsub, max_nt, k, bwd, fac, tvbuf, ybuf, z, nx, ny, s, c0, st)
    switch (groups) {
      case 1: ORAS_GEMM(1); break;
      case 2: ORAS_GEMM(2); break;
      case 3: ORAS_GEMM(3); break;
      case 4: ORAS_GEMM(4); break;
      case 5: ORAS_GEMM(5); break;
      case 6: ORAS_GEMM(6); break;
      case 7: ORAS_GEMM(7); break;
      default: ORAS_GEMM(8); break;
    }
#undef ORAS_GEMM
  }
}

}  // namespace

template <typename R, typename Z>
void launch_oras_apply(const OrasPlan& plan, const C<R>* fac, const C<R>* lca, C<R>* ybuf,
                       C<R>* tvbuf, const double2* v, const double* scale, Z* z, int nx, int ny,
                       int s, hipStream_t st, hipEvent_t* gemm_ev) {
  const int bs = 256;
  const dim3 grhs((unsigned)((plan.max_p * s + bs - 1) / bs), (unsigned)plan.nsub);
  const int nsteps = 2 * plan.max_sz - 1;
  for (int step = 0; step < nsteps; ++step) {
    const bool bwd = step >= plan.max_sz;
    const int k = bwd ? 2 * plan.max_sz - 2 - step : step;
    hipLaunchKernelGGL((plane_rhs_kernel<R>), grhs, dim3(bs), 0, st, plan.subs, k, bwd ? 1 : 0, lca,
                       ybuf, tvbuf, v, scale, nx, ny, s);
    if (gemm_ev) (void)hipEventRecord(gemm_ev[2 * step], st);
    gemm_dispatch<R, Z>(plan.subs, plan.nsub, plan.max_nt, k, bwd ? 1 : 0, fac, tvbuf, ybuf, z,
                        nx, ny, s, st);
    if (gemm_ev) (void)hipEventRecord(gemm_ev[2 * step + 1], st);
  }
}

template void launch_oras_apply<float, float2>(const OrasPlan&, const float2*, const float2*,
                                               float2*, float2*, const double2*, const double*,
                                               float2*, int, int, int, hipStream_t, hipEvent_t*);
template void launch_oras_apply<float, double2>(const OrasPlan&, const float2*, const float2*,
                                                float2*, float2*, const double2*, const double*,
                                                double2*, int, int, int, hipStream_t,
                                                hipEvent_t*);
template void launch_oras_apply<double, double2>(const OrasPlan&, const double2*, const double2*,
                                                 double2*, double2*, const double2*,
                                                 const double*, double2*, int, int, int,
                                                 hipStream_t, hipEvent_t*);

}  // namespace oras
