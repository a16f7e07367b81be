// Device factorisation of the ORAS local matrices B_j (paper sec. 2.2: the
// local matrices are factorised once at set-up; the paper uses a sparse
// direct solver, here the factorisation is rebuilt for the GPU).
//
// A box of sx x sy x sz nodes ordered plane by plane (z slowest) makes B_j
// block tridiagonal with p x p plane blocks (p = sx sy), because the
// 27-point stencil couples a plane only to its two neighbours.  Block
// elimination over the planes gives the Schur complements
//     S_0 = D_0,   S_k = D_k - L_k S_{k-1}^{-1} U_{k-1},
// and the factors kept are the explicit inverses S_k^{-1}.  A solve is then
// two sweeps of dense products (forward y_k = S_k^{-1}(r_k - L_k y_{k-1}),
// backward x_k = y_k - S_k^{-1} U_k x_{k+1}), which map onto MFMA.
//
// Every plane matrix is padded to P = ceil(p / 32) * 32 (identity on the pad)
// and stored as 32 x 32 tiles, tile (I, J) at ((I nt + J) * 1024); inside a
// tile, entry (r, c) sits at ((c / 4) * 32 + r) * 4 + c % 4, so four
// consecutive columns of 16 or 32 consecutive rows form one contiguous run
// (the operand fragment of a 16x16x4 MFMA, and a 4x4 register block).
//
// The inverse is formed in place by blocked Gauss-Jordan elimination with
// 32 x 32 pivot blocks (no pivoting; a zero or non-finite pivot is reported):
//     A_kk <- A_kk^{-1};  A_kJ <- A_kk^{-1} A_kJ;  A_IJ <- A_IJ - A_Ik A_kJ;
//     A_Ik <- -A_Ik A_kk^{-1}.
// The trailing update A_IJ -= A_Ik A_kJ, which carries almost all the work,
// runs on MFMA; the panel and pivot-block steps are small and use VALU.
#include "oras_internal.h"

namespace oras {

namespace {

__device__ inline long long tile_off(int I, int J, int nt) {
  return ((long long)I * nt + J) * (TILE * TILE);
}
__device__ inline int in_tile(int r, int c) { return ((c >> 2) * TILE + r) * 4 + (c & 3); }
__device__ inline long long mat_off(int row, int col, int nt) {
  return tile_off(row / TILE, col / TILE, nt) + in_tile(row % TILE, col % TILE);
}

template <typename T> __device__ inline T czero() { T z; z.x = 0; z.y = 0; return z; }
template <typename T> __device__ inline T cone() { T z; z.x = 1; z.y = 0; return z; }

template <typename R> struct Tiny;
template <> struct Tiny<float> { static constexpr float v = 1e-30f; };
template <> struct Tiny<double> { static constexpr double v = 1e-280; };

// T = S_{k-1}^{-1} U_{k-1}:  T[a, c] = sum_d Sinv[a, c - d] U[c - d, c], where
// U[c', c] couples node c' of plane k-1 to node c of plane k.
template <typename R>
__global__ void __launch_bounds__(256) schur_T_kernel(const SubDesc* subs, int k, const C<R>* fac,
                                                      C<R>* tbuf, const C<R>* lca) {
  using T = C<R>;
  const SubDesc sd = subs[blockIdx.z];
  if (k == 0 || k >= sd.sz) return;
  const int nt = sd.nt;
  const int I = blockIdx.y, J = blockIdx.x;
  if (I >= nt || J >= nt) return;
  const long long P2 = (long long)sd.P * sd.P;
  const T* Sinv = fac + sd.fac_off + (long long)(k - 1) * P2;
  T* Tm = tbuf + sd.t_off;
  const long long nbox = (long long)sd.sx * sd.sy * sd.sz;
  const T* L = lca + sd.lca_off;
  for (int q = 0; q < 4; ++q) {
    const int e = threadIdx.x + 256 * q;
    const int c4 = e >> 7, r = (e >> 2) & 31, cl = e & 3;
    const int a = I * TILE + r, c = J * TILE + c4 * 4 + cl;
    T acc = czero<T>();
    if (c < sd.p) {
      const int cx = c % sd.sx, cy = c / sd.sx;
      for (int dy = -1; dy <= 1; ++dy) {
        const int py = cy - dy;
        if (py < 0 || py >= sd.sy) continue;
        for (int dx = -1; dx <= 1; ++dx) {
          const int px = cx - dx;
          if (px < 0 || px >= sd.sx) continue;
          const long long node = ((long long)(k - 1) * sd.sy + py) * sd.sx + px;
          const T u = L[eidx(dx, dy, 1) * nbox + node];
          const T s = Sinv[mat_off(a, py * sd.sx + px, nt)];
          cfma(acc, s, u);
        }
      }
    }
    Tm[tile_off(I, J, nt) + e] = acc;
  }
}

// S_k = D_k - L_k T  (just D_k on the first plane), identity on the pad.
template <typename R>
__global__ void __launch_bounds__(256) build_S_kernel(const SubDesc* subs, int k, C<R>* fac,
                                                      const C<R>* tbuf, const C<R>* lca) {
  using T = C<R>;
  const SubDesc sd = subs[blockIdx.z];
  if (k >= sd.sz) return;
  const int nt = sd.nt;
  const int I = blockIdx.y, J = blockIdx.x;
  if (I >= nt || J >= nt) return;
  const long long P2 = (long long)sd.P * sd.P;
  T* S = fac + sd.fac_off + (long long)k * P2;
  const T* Tm = tbuf + sd.t_off;
  const long long nbox = (long long)sd.sx * sd.sy * sd.sz;
  const T* L = lca + sd.lca_off;
  for (int q = 0; q < 4; ++q) {
    const int e = threadIdx.x + 256 * q;
    const int c4 = e >> 7, r = (e >> 2) & 31, cl = e & 3;
    const int b = I * TILE + r, c = J * TILE + c4 * 4 + cl;
    T v = czero<T>();
    if (b >= sd.p || c >= sd.p) {
      if (b == c) v = cone<T>();
    } else {
      const int bx = b % sd.sx, by = b / sd.sx;
      const int cx = c % sd.sx, cy = c / sd.sx;
      const long long node = ((long long)k * sd.sy + by) * sd.sx + bx;
      const int dx = cx - bx, dy = cy - by;
      if (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1) v = L[eidx(dx, dy, 0) * nbox + node];
      if (k > 0) {
        for (int ey = -1; ey <= 1; ++ey) {
          const int qy = by + ey;
          if (qy < 0 || qy >= sd.sy) continue;
          for (int ex = -1; ex <= 1; ++ex) {
            const int qx = bx + ex;
            if (qx < 0 || qx >= sd.sx) continue;
            const T l = L[eidx(ex, ey, -1) * nbox + node];
            const T t = Tm[mat_off(qy * sd.sx + qx, c, nt)];
            cfms(v, l, t);
          }
        }
      }
    }
    S[tile_off(I, J, nt) + e] = v;
  }
}

// ---- tile helpers: 64 threads, thread (tr, tc) owns rows 4 tr.., cols 4 tc..
template <typename T>
__device__ inline void load_tile_lds(const T* g, T (*lds)[TILE + 1]) {
  for (int q = 0; q < 16; ++q) {
    const int e = threadIdx.x + 64 * q;
    const int c4 = e >> 7, r = (e >> 2) & 31, cl = e & 3;
    lds[r][c4 * 4 + cl] = g[e];
  }
}
// out(i, j) = sum_m X[4 tr + i][m] Y[m][4 tc + j]
template <typename T>
__device__ inline void tile_product(const T (*X)[TILE + 1], const T (*Y)[TILE + 1], T out[4][4]) {
  const int tr = threadIdx.x >> 3, tc = threadIdx.x & 7;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) out[i][j] = czero<T>();
  for (int m = 0; m < TILE; ++m) {
    T xv[4], yv[4];
    for (int i = 0; i < 4; ++i) xv[i] = X[4 * tr + i][m];
    for (int j = 0; j < 4; ++j) yv[j] = Y[m][4 * tc + j];
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) cfma(out[i][j], xv[i], yv[j]);
  }
}
// contiguous 16-entry run of the thread's 4x4 block inside a tile
__device__ inline int block_base() {
  const int tr = threadIdx.x >> 3, tc = threadIdx.x & 7;
  return (tc * TILE + tr * 4) * 4;
}

// A_kk <- A_kk^{-1} by unblocked Gauss-Jordan in LDS.
template <typename R>
__global__ void __launch_bounds__(256) gj_diag_kernel(const SubDesc* subs, int k, int kb,
                                                      C<R>* fac, int* status) {
  using T = C<R>;
  __shared__ T A[TILE][TILE + 1];
  __shared__ int bad;
  const SubDesc sd = subs[blockIdx.x];
  if (k >= sd.sz || kb >= sd.nt) return;
  const long long P2 = (long long)sd.P * sd.P;
  T* tile = fac + sd.fac_off + (long long)k * P2 + tile_off(kb, kb, sd.nt);
  for (int q = 0; q < 4; ++q) {
    const int e = threadIdx.x + 256 * q;
    const int c4 = e >> 7, r = (e >> 2) & 31, cl = e & 3;
    A[r][c4 * 4 + cl] = tile[e];
  }
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  for (int piv = 0; piv < TILE; ++piv) {
    const T p = A[piv][piv];
    const R mag = p.x * p.x + p.y * p.y;
    const bool ok = isfinite(p.x) && isfinite(p.y) && mag > Tiny<R>::v;
    T ip;
    {
      const R d = ok ? mag : (R)1;
      ip.x = p.x / d;
      ip.y = -p.y / d;
    }
    if (!ok && threadIdx.x == 0) bad = 1;
    __syncthreads();
    if (threadIdx.x < TILE && threadIdx.x != piv) {
      A[piv][threadIdx.x] = cmul(A[piv][threadIdx.x], ip);
    }
    __syncthreads();
    for (int q = 0; q < 4; ++q) {
      const int e = threadIdx.x + 256 * q;
      const int r = e >> 5, c = e & 31;
      if (r != piv && c != piv) {
        const T f = A[r][piv];
        const T g = A[piv][c];
        T v = A[r][c];
        cfms(v, f, g);
        A[r][c] = v;
      }
    }
    __syncthreads();
    if (threadIdx.x < TILE) {
      const int r = threadIdx.x;
      if (r != piv) {
        T v = cmul(A[r][piv], ip);
        v.x = -v.x;
        v.y = -v.y;
        A[r][piv] = v;
      } else {
        A[piv][piv] = ip;
      }
    }
    __syncthreads();
  }
  for (int q = 0; q < 4; ++q) {
    const int e = threadIdx.x + 256 * q;
    const int c4 = e >> 7, r = (e >> 2) & 31, cl = e & 3;
    tile[e] = A[r][c4 * 4 + cl];
  }
  if (threadIdx.x == 0 && bad) status[blockIdx.x] = 1;
}

// A_kJ <- A_kk^{-1} A_kJ   (J != kb)
template <typename R>
__global__ void __launch_bounds__(64) gj_rowpanel_kernel(const SubDesc* subs, int k, int kb,
                                                         C<R>* fac) {
  using T = C<R>;
  __shared__ T D[TILE][TILE + 1];
  __shared__ T B[TILE][TILE + 1];
  const SubDesc sd = subs[blockIdx.y];
  const int J = blockIdx.x;
  if (k >= sd.sz || kb >= sd.nt || J >= sd.nt || J == kb) return;
  T* base = fac + sd.fac_off + (long long)k * sd.P * sd.P;
  load_tile_lds(base + tile_off(kb, kb, sd.nt), D);
  T* dst = base + tile_off(kb, J, sd.nt);
  load_tile_lds(dst, B);
  __syncthreads();
  T out[4][4];
  tile_product(D, B, out);
  const int o = block_base();
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) dst[o + i * 4 + j] = out[i][j];
}

// A_IJ <- A_IJ - A_Ik A_kJ   (I, J != kb) on MFMA, one wave per 32 x 32 tile.
// Work-group ids are mapped so that all tiles of one subdomain run on the same
// XCD and read the pivot row and column panels from its L2.
constexpr int NXCD = 8;
__device__ inline void tile_map(int items, int& sub, int& item) {
  const int b = blockIdx.x, r = b / NXCD;
  sub = (r / items) * NXCD + b % NXCD;
  item = r % items;
}

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename R> struct GjUpdate;

// Complex FP32 on the 32x32x2 instruction.  The three tiles are fetched
// together up front (A_Ik and A_kJ into LDS, A_IJ into registers), so a wave
// waits for memory once.  A_Ik rows come from the tile layout (lane l: row
// l % 32, entries 2 (l / 32), 2 (l / 32) + 1 of each 4-column run); B = A_kJ
// is read per lane as the complex entry (k, col) and split into [Br | Bi] and
// [-Bi | Br] by lane parity.  Real and imaginary A parts accumulate
// separately (four independent chains).
template <> struct GjUpdate<float> {
  static __device__ void run(float2* __restrict__ C, const float2* __restrict__ X,
                             const float2* __restrict__ Y) {
    __shared__ float4 sX[512], sY[512];
    const int lane = threadIdx.x, rr = lane & 31, h = lane >> 5;
    const bool odd = (rr & 1) != 0;
    float* Cf = reinterpret_cast<float*>(C);
    float4 xr[8], yr[8];
    float cv[2][16];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      xr[i] = reinterpret_cast<const float4*>(X)[i * 64 + lane];
      yr[i] = reinterpret_cast<const float4*>(Y)[i * 64 + lane];
    }
    // accumulator item i of lane l: row 8 (i / 4) + 4 (l / 32) + i % 4, real column l % 32
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int row = 8 * (i / 4) + 4 * h + (i % 4);
#pragma unroll
      for (int b = 0; b < 2; ++b) cv[b][i] = Cf[2 * in_tile(row, 16 * b + (rr >> 1)) + (rr & 1)];
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      sX[i * 64 + lane] = xr[i];
      sY[i * 64 + lane] = yr[i];
    }
    __syncthreads();
    const float2* Ys = reinterpret_cast<const float2*>(sY);
    f32x16 acc[2][2];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        acc[b][0][j] = 0.f;
        acc[b][1][j] = 0.f;
      }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const float4 a = sX[q * 64 + rr * 2 + h];
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const float ar = e ? a.z : a.x, ai = e ? a.w : a.y;
        const int kr = 4 * q + 2 * h + e;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const float2 v = Ys[in_tile(kr, 16 * b + (rr >> 1))];
          const float b1 = odd ? v.y : v.x, b2 = odd ? v.x : -v.y;
          acc[b][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, b1, acc[b][0], 0, 0, 0);
          acc[b][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai, b2, acc[b][1], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int row = 8 * (i / 4) + 4 * h + (i % 4);
#pragma unroll
      for (int b = 0; b < 2; ++b)
        Cf[2 * in_tile(row, 16 * b + (rr >> 1)) + (rr & 1)] = cv[b][i] - (acc[b][0][i] + acc[b][1][i]);
    }
  }
};

// Complex FP64 on the 16x16x4 FP64 instruction (operands A[row = l % 16][k =
// l / 16], B[k = l / 16][col = l % 16]; result item t of lane l is row
// l / 16 + 4 t): two 16-row halves x four 8-column groups, tiles fetched up
// front as in the FP32 form.
template <> struct GjUpdate<double> {
  static __device__ void run(double2* __restrict__ C, const double2* __restrict__ X,
                             const double2* __restrict__ Y) {
    __shared__ double2 sX[1024], sY[1024];
    const int lane = threadIdx.x, m = lane & 15, kk = lane >> 4;
    const bool odd = (m & 1) != 0;
    double* Cd = reinterpret_cast<double*>(C);
    double2 xr[16], yr[16];
    double cv[2][4][4];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      xr[i] = X[i * 64 + lane];
      yr[i] = Y[i * 64 + lane];
    }
#pragma unroll
    for (int rs = 0; rs < 2; ++rs)
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int ns = 0; ns < 4; ++ns)
          cv[rs][t][ns] = Cd[2 * in_tile(rs * 16 + kk + 4 * t, 8 * ns + (m >> 1)) + (m & 1)];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      sX[i * 64 + lane] = xr[i];
      sY[i * 64 + lane] = yr[i];
    }
    __syncthreads();
    f64x4 acc[2][4];
#pragma unroll
    for (int rs = 0; rs < 2; ++rs)
#pragma unroll
      for (int ns = 0; ns < 4; ++ns) acc[rs][ns] = f64x4{0, 0, 0, 0};
#pragma unroll 2
    for (int q = 0; q < 8; ++q) {
      const double2 a0 = sX[(q * TILE + m) * 4 + kk];
      const double2 a1 = sX[(q * TILE + 16 + m) * 4 + kk];
      const int kr = 4 * q + kk;
#pragma unroll
      for (int ns = 0; ns < 4; ++ns) {
        const double2 v = sY[in_tile(kr, 8 * ns + (m >> 1))];
        const double b1 = odd ? v.y : v.x, b2 = odd ? v.x : -v.y;
        acc[0][ns] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0.x, b1, acc[0][ns], 0, 0, 0);
        acc[0][ns] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0.y, b2, acc[0][ns], 0, 0, 0);
        acc[1][ns] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1.x, b1, acc[1][ns], 0, 0, 0);
        acc[1][ns] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1.y, b2, acc[1][ns], 0, 0, 0);
      }
    }
#pragma unroll
    for (int rs = 0; rs < 2; ++rs)
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int ns = 0; ns < 4; ++ns)
          Cd[2 * in_tile(rs * 16 + kk + 4 * t, 8 * ns + (m >> 1)) + (m & 1)] =
              cv[rs][t][ns] - acc[rs][ns][t];
  }
};

template <typename R>
__global__ void __launch_bounds__(64) gj_update_kernel(const SubDesc* subs, int nsub, int max_nt,
                                                       int k, int kb, C<R>* fac) {
  int sub, item;
  tile_map(max_nt * max_nt, sub, item);
  if (sub >= nsub) return;
  const SubDesc sd = subs[sub];
  const int I = item / max_nt, J = item % max_nt;
  if (k >= sd.sz || kb >= sd.nt || I >= sd.nt || J >= sd.nt || I == kb || J == kb) return;
  C<R>* base = fac + sd.fac_off + (long long)k * sd.P * sd.P;
  GjUpdate<R>::run(base + tile_off(I, J, sd.nt), base + tile_off(I, kb, sd.nt),
                   base + tile_off(kb, J, sd.nt));
}

// A_Ik <- -A_Ik A_kk^{-1}   (I != kb)
template <typename R>
__global__ void __launch_bounds__(64) gj_colpanel_kernel(const SubDesc* subs, int k, int kb,
                                                         C<R>* fac) {
  using T = C<R>;
  __shared__ T X[TILE][TILE + 1];
  __shared__ T D[TILE][TILE + 1];
  const SubDesc sd = subs[blockIdx.y];
  const int I = blockIdx.x;
  if (k >= sd.sz || kb >= sd.nt || I >= sd.nt || I == kb) return;
  T* base = fac + sd.fac_off + (long long)k * sd.P * sd.P;
  T* dst = base + tile_off(I, kb, sd.nt);
  load_tile_lds(dst, X);
  load_tile_lds(base + tile_off(kb, kb, sd.nt), D);
  __syncthreads();
  T out[4][4];
  tile_product(X, D, out);
  const int o = block_base();
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      T v = out[i][j];
      v.x = -v.x;
      v.y = -v.y;
      dst[o + i * 4 + j] = v;
    }
}

}  // namespace

template <typename R>
void launch_factor_plane(const SubDesc* subs_dev, int nsub, int k, int max_nt, C<R>* fac,
                         C<R>* tbuf, const C<R>* lca, int* status, hipStream_t st) {
  const dim3 g2(max_nt, max_nt, nsub);
  const int nsub8 = (nsub + NXCD - 1) / NXCD * NXCD;
  if (k > 0)
    hipLaunchKernelGGL((schur_T_kernel<R>), g2, dim3(256), 0, st, subs_dev, k, fac, tbuf, lca);
  hipLaunchKernelGGL((build_S_kernel<R>), g2, dim3(256), 0, st, subs_dev, k, fac, tbuf, lca);
  for (int kb = 0; kb < max_nt; ++kb) {
    hipLaunchKernelGGL((gj_diag_kernel<R>), dim3(nsub), dim3(256), 0, st, subs_dev, k, kb, fac,
                       status);
    hipLaunchKernelGGL((gj_rowpanel_kernel<R>), dim3(max_nt, nsub), dim3(64), 0, st, subs_dev, k,
                       kb, fac);
    hipLaunchKernelGGL((gj_update_kernel<R>), dim3((unsigned)(nsub8 * max_nt * max_nt)), dim3(64),
                       0, st, subs_dev, nsub, max_nt, k, kb, fac);
    hipLaunchKernelGGL((gj_colpanel_kernel<R>), dim3(max_nt, nsub), dim3(64), 0, st, subs_dev, k,
                       kb, fac);
  }
}

template void launch_factor_plane<float>(const SubDesc*, int, int, int, float2*, float2*,
                                         const float2*, int*, hipStream_t);
template void launch_factor_plane<double>(const SubDesc*, int, int, int, double2*, double2*,
                                          const double2*, int*, hipStream_t);

}  // namespace oras
