// Block low-rank (BLR) plane inverses for the ORAS local solves (paper sec. 3:
// the local factors in BLR form with a threshold eps_BLR; Table 4).
//
// The factorisation leaves every plane inverse S_k^{-1} dense.  Compression
// cuts the plane into patches (rectangles of at most BLR_PMAX x BLR_PMAX
// nodes: along x ceil(sx / pmax) parts by floor split, likewise along y) and
// replaces every off-diagonal patch block by U V from a cross approximation
// with complete pivoting, stopped once the largest residual entry is at most
// eps times the plane's largest entry, so that bound holds for every entry of
// the error.  A block whose rank would pass b_I b_J / (b_I + b_J) (where the
// product costs as much as the block) stays dense, as do diagonal blocks.
//
// One plane step of the apply, for all subdomains:
//   * the right-hand side t is written row-major into rows 0..p-1 of the
//     subdomain's part of the operand buffer;
//   * projection: for every column patch J, T_J = V_J t_J (V_J: the V of the
//     patch's low-rank blocks, stacked) into further rows of that buffer;
//   * expansion: for every row patch I,
//         y_I = [S_II | S_IJ (dense blocks) | U_IJ (low-rank)] [t_I; t_J; T_IJ],
//     whose K operand rows are gathered through an address list; the
//     epilogue stores the plane rows and, on final planes, the owned nodes
//     (the same restricted prolongation as the dense substitution).
// Both are gather GEMMs on MFMA with the stored operand in [k / 4][row][k % 4]
// order.  Compression runs twice: a first pass finds the ranks, the host lays
// out the operands, and a second pass (the same deterministic kernel) writes
// them.
#include <algorithm>
#include <climits>

#include "oras_internal.h"

namespace oras {

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int NXCD = 8;

__device__ inline bool plane_active(const SubDesc& sd, int k, int bwd) {
  return bwd ? (k <= sd.sz - 2 && k >= sd.olo[2] - sd.lo[2]) : (k < sd.sz);
}

// Patch I of an sx x sy plane with an npx x npy patch grid.
__device__ inline void patch_box(int sx, int sy, int npx, int npy, int I, int& x0, int& w, int& y0,
                                 int& h) {
  const int px = I % npx, py = I / npx;
  x0 = px * sx / npx;
  w = (px + 1) * sx / npx - x0;
  y0 = py * sy / npy;
  h = (py + 1) * sy / npy - y0;
}

// Entry (row, col) of a plane inverse in the factor tile layout.
template <typename T>
__device__ inline T fac_at(const T* S, int nt, int row, int col) {
  const int r = row & 31, c = col & 31;
  return S[((long long)(row >> 5) * nt + (col >> 5)) * 1024 + ((c >> 2) * 32 + r) * 4 + (c & 3)];
}

template <typename T> __device__ inline T cdivT(T a, T b) {
  const auto d = b.x * b.x + b.y * b.y;
  T q;
  q.x = (a.x * b.x + a.y * b.y) / d;
  q.y = (a.y * b.x - a.x * b.y) / d;
  return q;
}

// --------------------------------------------------------- largest entry --
template <typename R>
__global__ void __launch_bounds__(256)
plane_max_kernel(const SubDesc* __restrict__ subs, int max_sz, const C<R>* __restrict__ fac,
                 double* __restrict__ smax) {
  const int sub = blockIdx.x / max_sz, k = blockIdx.x % max_sz;
  const SubDesc sd = subs[sub];
  if (k >= sd.sz) return;
  const C<R>* S = fac + sd.fac_off + (long long)k * sd.P * sd.P;
  const long long tot = (long long)sd.P * sd.P;
  double best = 0.0;
  for (long long e = threadIdx.x; e < tot; e += blockDim.x) {
    const int t = (int)(e >> 10), w = (int)(e & 1023);
    const int row = (t / sd.nt) * 32 + ((w >> 2) & 31);
    const int col = (t % sd.nt) * 32 + (w >> 7) * 4 + (w & 3);
    if (row < sd.p && col < sd.p) {
      const C<R> z = S[e];
      best = fmax(best, (double)z.x * z.x + (double)z.y * z.y);
    }
  }
  __shared__ double red[256];
  red[threadIdx.x] = best;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) smax[(long long)sub * max_sz + k] = sqrt(red[0]);
}

// ----------------------------------------------------------- compression --
// One work-group per patch block; thread t holds entries e = t + 256 j
// (row-major in the block, j < 16).  Each step finds the first largest
// |R_ab| (modulus squared in the factor precision, ties to the smaller
// row-major position), stops when it is at most tol, or when the rank cap is
// reached (dense), and otherwise subtracts u v with u = R[:, b],
// v = R[a, :] / R_ab.
constexpr int CT = 256;
constexpr int CPER = (BLR_PMAX * BLR_PMAX * BLR_PMAX * BLR_PMAX + CT - 1) / CT;

template <typename R, bool WRITE>
__global__ void __launch_bounds__(CT)
compress_kernel(const SubDesc* __restrict__ subs, const BlrSub* __restrict__ bsubs,
                const BlrBlock* __restrict__ blocks, long long nblocks,
                const C<R>* __restrict__ fac, const double* __restrict__ smax, int max_sz,
                double eps, int* __restrict__ rank_out, C<R>* __restrict__ astore,
                int* __restrict__ err) {
  using T = C<R>;
  const long long bid = blockIdx.x;
  if (bid >= nblocks) return;
  const BlrBlock blk = blocks[bid];
  const SubDesc sd = subs[blk.sub];
  const BlrSub bs = bsubs[blk.sub];
  int xi, wi, yi, hi, xj, wj, yj, hj;
  patch_box(sd.sx, sd.sy, bs.npx, bs.npy, blk.I, xi, wi, yi, hi);
  patch_box(sd.sx, sd.sy, bs.npx, bs.npy, blk.J, xj, wj, yj, hj);
  const int bI = wi * hi, bJ = wj * hj, nent = bI * bJ;
  const T* S = fac + sd.fac_off + (long long)blk.k * sd.P * sd.P;
  const int tid = threadIdx.x;
  auto load = [&](int e) {
    const int a = e / bJ, b = e % bJ;
    const int qa = (yi + a / wi) * sd.sx + xi + a % wi;
    const int qb = (yj + b / wj) * sd.sx + xj + b % wj;
    return fac_at(S, sd.nt, qa, qb);
  };
  // expansion operand of patch I: entry (row a, column e_koff + kk), 64-row stride
  auto e_store = [&](int a, int kk, T v) {
    astore[blk.e_off + ((long long)(kk >> 2) * 64 + a) * 4 + (kk & 3)] = v;
  };
  if (blk.I == blk.J) {
    if (WRITE) {
      for (int e = tid; e < nent; e += CT) e_store(e / bJ, blk.e_koff + e % bJ, load(e));
    } else if (tid == 0) {
      rank_out[bid] = -1;
    }
    return;
  }
  T Rv[CPER];
#pragma unroll
  for (int j = 0; j < CPER; ++j) {
    const int e = tid + CT * j;
    Rv[j] = e < nent ? load(e) : mk<R>(0, 0);
  }
  const R tol = (R)(eps * smax[(long long)blk.sub * max_sz + blk.k]);
  const R tol2 = tol * tol;
  const int cap = (bI * bJ) / (bI + bJ);
  __shared__ T u_s[BLR_PMAX * BLR_PMAX], vr_s[BLR_PMAX * BLR_PMAX], vn_s[BLR_PMAX * BLR_PMAX];
  __shared__ R red_v[CT / 64];
  __shared__ int red_i[CT / 64];
  int rank = 0;
  bool dense = false;
  for (;;) {
    R best = (R)-1;
    int bi = INT_MAX;
#pragma unroll
    for (int j = 0; j < CPER; ++j) {
      const int e = tid + CT * j;
      if (e < nent) {
        const R m = rfma(Rv[j].x, Rv[j].x, Rv[j].y * Rv[j].y);
        if (m > best) {
          best = m;
          bi = e;
        }
      }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      const R ob = __shfl_xor(best, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
      }
    }
    if ((tid & 63) == 0) {
      red_v[tid >> 6] = best;
      red_i[tid >> 6] = bi;
    }
    __syncthreads();
    best = red_v[0];
    bi = red_i[0];
#pragma unroll
    for (int w = 1; w < CT / 64; ++w)
      if (red_v[w] > best || (red_v[w] == best && red_i[w] < bi)) {
        best = red_v[w];
        bi = red_i[w];
      }
    if (!(best > tol2)) break;
    if (rank == cap) {
      dense = true;
      break;
    }
    const int as = bi / bJ, bsel = bi % bJ;
#pragma unroll
    for (int j = 0; j < CPER; ++j) {
      const int e = tid + CT * j;
      if (e < nent) {
        const int a = e / bJ, b = e % bJ;
        if (b == bsel) u_s[a] = Rv[j];
        if (a == as) vr_s[b] = Rv[j];
      }
    }
    __syncthreads();
    if (tid < bJ) vn_s[tid] = cdivT(vr_s[tid], vr_s[bsel]);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < CPER; ++j) {
      const int e = tid + CT * j;
      if (e < nent) cfms(Rv[j], u_s[e / bJ], vn_s[e % bJ]);
    }
    if (WRITE && rank < blk.rank) {
      if (tid < bI) e_store(tid, blk.e_koff + rank, u_s[tid]);
      if (tid < bJ)
        astore[blk.p_off + ((long long)(tid >> 2) * blk.p_mpad + blk.p_row + rank) * 4 + (tid & 3)] =
            vn_s[tid];
    }
    ++rank;
    __syncthreads();
  }
  const int result = dense ? -1 : rank;
  if (!WRITE) {
    if (tid == 0) rank_out[bid] = result;
    return;
  }
  if (result != blk.rank) {
    if (tid == 0) err[0] = 1;
    return;
  }
  if (dense)
    for (int e = tid; e < nent; e += CT) e_store(e / bJ, blk.e_koff + e % bJ, load(e));
}

// ------------------------------------------------------ right-hand side --
// t rows of every subdomain (row-major, pad16(s) columns): forward
// scale * v - L_k y_{k-1}, backward U_k x_{k+1}.
template <typename R>
__global__ void blr_rhs_kernel(const SubDesc* __restrict__ subs, const BlrSub* __restrict__ bsubs,
                               int k, int bwd, const C<R>* __restrict__ lca,
                               const C<R>* __restrict__ ybuf, C<R>* __restrict__ bt,
                               const double2* __restrict__ v, const double* __restrict__ scale,
                               int nx, int ny, int s, int s16) {
  const SubDesc sd = subs[blockIdx.y];
  if (!plane_active(sd, k, bwd)) return;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)sd.p * s) return;
  const int q = (int)(idx / s), c = (int)(idx % s);
  const int qx = q % sd.sx, qy = q / sd.sx;
  using T = C<R>;
  T t = mk<R>(0, 0);
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
    // couplings leaving the box are exact zeros in the local coefficients
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
      const int py = min(max(qy + dy, 0), sd.sy - 1);
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int px = min(max(qx + dx, 0), sd.sx - 1);
        const T l = L[eidx(dx, dy, ez) * nbox + node];
        const T y = Yn[(long long)(py * sd.sx + px) * s + c];
        if (bwd) cfma(t, l, y);
        else cfms(t, l, y);
      }
    }
  }
  bt[(bsubs[blockIdx.y].bt_off + q) * s16 + c] = t;
}

// --------------------------------------------------------- gather GEMMs --
// Work-group id -> (item, column group), with the items ordered so that every
// subdomain's items sit on one XCD.
__device__ inline bool item_map(int nitems, int ncg, int& it, int& cg) {
  const int b = blockIdx.x, r = b / NXCD;
  it = (r / ncg) * NXCD + b % NXCD;
  cg = r % ncg;
  return it < nitems;
}

// Operand-buffer row of the item's k-th operand row.  Projection: node k of
// the patch, as an offset from the patch's first node (its first node beyond
// the patch, where the stored operand column is zero); expansion: from the
// address list.
template <int MODE>
__device__ inline int b_row(const BlrItem& item, const int* addr, int w, int bsz, int sx, int kap) {
  if (MODE == 0) {
    const int l = kap < bsz ? kap : 0;
    return (l / w) * sx + l % w;
  }
  return addr[item.addr_off + kap];
}

// Complex FP32: 32x32x2 MFMA, RT tiles of 32 rows x 32 columns per wave.
template <int RT, int MODE, typename Z>
__global__ void __launch_bounds__(64)
blr_gemm_f32_kernel(const SubDesc* __restrict__ subs, const BlrSub* __restrict__ bsubs,
                    const BlrItem* __restrict__ items, int nitems, int ncg, int k, int bwd,
                    const float2* __restrict__ astore, const int* __restrict__ addr,
                    float2* __restrict__ bt, float2* __restrict__ ybuf, Z* __restrict__ z,
                    int nx, int ny, int s, int s16) {
  using ZR = typename std::conditional<sizeof(Z) == 8, float, double>::type;
  int it, cg;
  if (!item_map(nitems, ncg, it, cg)) return;
  const BlrItem item = items[it];
  if (item.sub < 0) return;
  const SubDesc sd = subs[item.sub];
  if (!plane_active(sd, k, bwd)) return;
  const BlrSub bs = bsubs[item.sub];
  int x0, w, y0, hh;
  patch_box(sd.sx, sd.sy, bs.npx, bs.npy, item.patch, x0, w, y0, hh);
  const int bsz = w * hh;
  const int origin = y0 * sd.sx + x0;           // plane row of the patch's first node
  const float* btf = reinterpret_cast<const float*>(bt + bs.bt_off * s16);
  const float4* A = reinterpret_cast<const float4*>(astore + item.a_off);
  const int lane = threadIdx.x, rr = lane & 31, h = lane >> 5;
  const bool odd = (rr & 1) != 0;
  const int c0 = 32 * cg;
  int colf[2];
  bool colok[2];
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
    const int col = c0 + 16 * nb + (rr >> 1);
    colok[nb] = col < s16;
    colf[nb] = 2 * col + (rr & 1);
  }
  f32x16 acc[RT][2][2];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        acc[rt][nb][0][j] = 0.f;
        acc[rt][nb][1][j] = 0.f;
      }
  const int nkq = item.K >> 2;
#pragma unroll 2
  for (int kq = 0; kq < nkq; ++kq) {
    int row[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int kap = 4 * kq + 2 * h + e;
      row[e] = MODE == 0 ? origin + b_row<0>(item, addr, w, bsz, sd.sx, kap)
                         : b_row<1>(item, addr, w, bsz, sd.sx, kap);
    }
    float bv[2][2];
#pragma unroll
    for (int e = 0; e < 2; ++e)
#pragma unroll
      for (int nb = 0; nb < 2; ++nb)
        bv[e][nb] = colok[nb] ? btf[(long long)row[e] * 2 * s16 + colf[nb]] : 0.f;
    float4 a[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
      a[rt] = A[((long long)kq * item.mpad + item.row0 + 32 * rt + rr) * 2 + h];
#pragma unroll
    for (int e = 0; e < 2; ++e)
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) {
        const float b1 = bv[e][nb];
        const float sw = __int_as_float(__builtin_amdgcn_update_dpp(
            __float_as_int(b1), __float_as_int(b1), 0xB1, 0xF, 0xF, false));
        const float b2 = odd ? sw : -sw;
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
          const float ar = e ? a[rt].z : a[rt].x, ai = e ? a[rt].w : a[rt].y;
          acc[rt][nb][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, b1, acc[rt][nb][0], 0, 0, 0);
          acc[rt][nb][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai, b2, acc[rt][nb][1], 0, 0, 0);
        }
      }
  }
  // accumulator item i of lane l: row 8 (i / 4) + 4 (l / 32) + i % 4, real column l % 32
  if (MODE == 0) {
    float* Tf = reinterpret_cast<float*>(bt + (bs.bt_off + item.out_row) * s16);
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int lr = 32 * rt + 8 * (i / 4) + 4 * h + (i % 4);
        if (lr >= item.rows) continue;
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
          const int col = c0 + 16 * nb + (rr >> 1);
          if (col >= s) continue;
          Tf[(long long)lr * 2 * s16 + colf[nb]] = acc[rt][nb][0][i] + acc[rt][nb][1][i];
        }
      }
    return;
  }
  const bool final_plane = bwd || (k == sd.sz - 1);
  float* Yk = reinterpret_cast<float*>(ybuf + (sd.y_off + (long long)k * sd.P) * s);
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int l = 32 * rt + 8 * (i / 4) + 4 * h + (i % 4);
      if (l >= bsz) continue;
      const int qx = x0 + l % w, qy = y0 + l / w;
      float* yr = Yk + (long long)(qy * sd.sx + qx) * 2 * s;
      long long zoff = -1;
      if (final_plane) {
        const int gx = sd.lo[0] + qx, gy = sd.lo[1] + qy, gz = sd.lo[2] + k;
        if (gx >= sd.olo[0] && gx < sd.ohi[0] && gy >= sd.olo[1] && gy < sd.ohi[1] &&
            gz >= sd.olo[2] && gz < sd.ohi[2])
          zoff = (((long long)gz * ny + gy) * nx + gx) * s;
      }
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) {
        const int col = c0 + 16 * nb + (rr >> 1);
        if (col >= s) continue;
        const int fi = 2 * col + (rr & 1);
        float val = acc[rt][nb][0][i] + acc[rt][nb][1][i];
        if (bwd) val = yr[fi] - val;
        yr[fi] = val;
        if (zoff >= 0) reinterpret_cast<ZR*>(z + zoff)[fi] = (ZR)val;
      }
    }
}

// Complex FP64: 16x16x4 MFMA, RG groups of 16 rows x 16 columns per wave.
// A[row = lane % 16][k = lane / 16], B[k = lane / 16][col = lane % 16];
// result item t of lane l is row l / 16 + 4 t, column l % 16.
template <int RG, int MODE>
__global__ void __launch_bounds__(64)
blr_gemm_f64_kernel(const SubDesc* __restrict__ subs, const BlrSub* __restrict__ bsubs,
                    const BlrItem* __restrict__ items, int nitems, int ncg, int k, int bwd,
                    const double2* __restrict__ astore, const int* __restrict__ addr,
                    double2* __restrict__ bt, double2* __restrict__ ybuf,
                    double2* __restrict__ z, int nx, int ny, int s, int s16) {
  int it, cg;
  if (!item_map(nitems, ncg, it, cg)) return;
  const BlrItem item = items[it];
  if (item.sub < 0) return;
  const SubDesc sd = subs[item.sub];
  if (!plane_active(sd, k, bwd)) return;
  const BlrSub bs = bsubs[item.sub];
  int x0, w, y0, hh;
  patch_box(sd.sx, sd.sy, bs.npx, bs.npy, item.patch, x0, w, y0, hh);
  const int bsz = w * hh;
  const int origin = y0 * sd.sx + x0;
  const double2* btc = bt + bs.bt_off * s16;
  const double2* A = astore + item.a_off;
  const int lane = threadIdx.x, m = lane & 15, kk = lane >> 4;
  const int bn = m >> 1;
  const bool im = (m & 1) != 0;
  const int c0 = 16 * cg;
  f64x4 acc[RG][2];
#pragma unroll
  for (int rg = 0; rg < RG; ++rg)
#pragma unroll
    for (int ns = 0; ns < 2; ++ns) acc[rg][ns] = f64x4{0, 0, 0, 0};
  const int nkq = item.K >> 2;
  for (int kq = 0; kq < nkq; ++kq) {
    const int kap = 4 * kq + kk;
    const int row = MODE == 0 ? origin + b_row<0>(item, addr, w, bsz, sd.sx, kap)
                              : b_row<1>(item, addr, w, bsz, sd.sx, kap);
#pragma unroll
    for (int ns = 0; ns < 2; ++ns) {
      const int col = c0 + 8 * ns + bn;
      const double2 bv = col < s16 ? btc[(long long)row * s16 + col] : make_double2(0.0, 0.0);
      const double b1 = im ? bv.y : bv.x;
      const double b2 = im ? bv.x : -bv.y;
#pragma unroll
      for (int rg = 0; rg < RG; ++rg) {
        const double2 a = A[((long long)kq * item.mpad + item.row0 + 16 * rg + m) * 4 + kk];
        acc[rg][ns] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b1, acc[rg][ns], 0, 0, 0);
        acc[rg][ns] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b2, acc[rg][ns], 0, 0, 0);
      }
    }
  }
  if (MODE == 0) {
    double* Tf = reinterpret_cast<double*>(bt + (bs.bt_off + item.out_row) * s16);
#pragma unroll
    for (int rg = 0; rg < RG; ++rg)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int lr = 16 * rg + kk + 4 * t;
        if (lr >= item.rows) continue;
#pragma unroll
        for (int ns = 0; ns < 2; ++ns) {
          const int col = c0 + 8 * ns + bn;
          if (col >= s) continue;
          Tf[(long long)lr * 2 * s16 + 2 * col + (im ? 1 : 0)] = acc[rg][ns][t];
        }
      }
    return;
  }
  const bool final_plane = bwd || (k == sd.sz - 1);
  double* Yk = reinterpret_cast<double*>(ybuf + (sd.y_off + (long long)k * sd.P) * s);
#pragma unroll
  for (int rg = 0; rg < RG; ++rg)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int l = 16 * rg + kk + 4 * t;
      if (l >= bsz) continue;
      const int qx = x0 + l % w, qy = y0 + l / w;
      double* yr = Yk + (long long)(qy * sd.sx + qx) * 2 * s;
      long long zoff = -1;
      if (final_plane) {
        const int gx = sd.lo[0] + qx, gy = sd.lo[1] + qy, gz = sd.lo[2] + k;
        if (gx >= sd.olo[0] && gx < sd.ohi[0] && gy >= sd.olo[1] && gy < sd.ohi[1] &&
            gz >= sd.olo[2] && gz < sd.ohi[2])
          zoff = (((long long)gz * ny + gy) * nx + gx) * s;
      }
#pragma unroll
      for (int ns = 0; ns < 2; ++ns) {
        const int col = c0 + 8 * ns + bn;
        if (col >= s) continue;
        const int fi = 2 * col + (im ? 1 : 0);
        double val = acc[rg][ns][t];
        if (bwd) val = yr[fi] - val;
        yr[fi] = val;
        if (zoff >= 0) reinterpret_cast<double*>(z + zoff)[fi] = val;
      }
    }
}

template <typename R, typename Z> struct BlrStep;
template <typename Z> struct BlrStep<float, Z> {
  static void gemm(const BlrApply& pl, int k, int bwd, const float2* astore, float2* bt,
                   float2* ybuf, Z* z, int nx, int ny, int s, int s16, hipStream_t st) {
    const int ncg = (s + 31) / 32;
    if (pl.p_count[k] > 0)
      hipLaunchKernelGGL((blr_gemm_f32_kernel<1, 0, Z>), dim3((unsigned)(pl.p_count[k] * ncg)),
                         dim3(64), 0, st, pl.subs, pl.bsubs, pl.items + pl.p_first[k],
                         pl.p_count[k], ncg, k, bwd, astore, pl.addr, bt, ybuf, z, nx, ny, s, s16);
    hipLaunchKernelGGL((blr_gemm_f32_kernel<2, 1, Z>), dim3((unsigned)(pl.e_count[k] * ncg)),
                       dim3(64), 0, st, pl.subs, pl.bsubs, pl.items + pl.e_first[k],
                       pl.e_count[k], ncg, k, bwd, astore, pl.addr, bt, ybuf, z, nx, ny, s, s16);
  }
};
template <> struct BlrStep<double, double2> {
  static void gemm(const BlrApply& pl, int k, int bwd, const double2* astore, double2* bt,
                   double2* ybuf, double2* z, int nx, int ny, int s, int s16, hipStream_t st) {
    const int ncg = (s + 15) / 16;
    if (pl.p_count[k] > 0)
      hipLaunchKernelGGL((blr_gemm_f64_kernel<2, 0>), dim3((unsigned)(pl.p_count[k] * ncg)),
                         dim3(64), 0, st, pl.subs, pl.bsubs, pl.items + pl.p_first[k],
                         pl.p_count[k], ncg, k, bwd, astore, pl.addr, bt, ybuf, z, nx, ny, s, s16);
    hipLaunchKernelGGL((blr_gemm_f64_kernel<4, 1>), dim3((unsigned)(pl.e_count[k] * ncg)),
                       dim3(64), 0, st, pl.subs, pl.bsubs, pl.items + pl.e_first[k],
                       pl.e_count[k], ncg, k, bwd, astore, pl.addr, bt, ybuf, z, nx, ny, s, s16);
  }
};

}  // namespace

template <typename R>
void launch_blr_plane_max(const SubDesc* subs, int nsub, int max_sz, const C<R>* fac,
                          double* smax, hipStream_t st) {
  hipLaunchKernelGGL((plane_max_kernel<R>), dim3((unsigned)(nsub * max_sz)), dim3(256), 0, st, subs,
                     max_sz, fac, smax);
}

template <typename R>
void launch_blr_compress(const SubDesc* subs, const BlrSub* bsubs, const BlrBlock* blocks,
                         long long nblocks, const C<R>* fac, const double* smax, int max_sz,
                         double eps, int* rank_out, C<R>* astore, int* err, hipStream_t st) {
  if (nblocks <= 0) return;
  if (astore)
    hipLaunchKernelGGL((compress_kernel<R, true>), dim3((unsigned)nblocks), dim3(CT), 0, st, subs,
                       bsubs, blocks, nblocks, fac, smax, max_sz, eps, rank_out, astore, err);
  else
    hipLaunchKernelGGL((compress_kernel<R, false>), dim3((unsigned)nblocks), dim3(CT), 0, st, subs,
                       bsubs, blocks, nblocks, fac, smax, max_sz, eps, rank_out, astore, err);
}

template <typename R, typename Z>
void launch_oras_apply_blr(const BlrApply& pl, const C<R>* astore, const C<R>* lca, C<R>* ybuf,
                           C<R>* bt, const double2* v, const double* scale, Z* z, int nx, int ny,
                           int s, hipStream_t st, hipEvent_t* gemm_ev) {
  const int s16 = (int)pad16(s);
  const int nsteps = 2 * pl.max_sz - 1;
  const int bs = 256;
  const dim3 grhs((unsigned)((pl.max_p * s + bs - 1) / bs), (unsigned)pl.nsub);
  for (int step = 0; step < nsteps; ++step) {
    const int bwd = step >= pl.max_sz ? 1 : 0;
    const int k = bwd ? 2 * pl.max_sz - 2 - step : step;
    hipLaunchKernelGGL((blr_rhs_kernel<R>), grhs, dim3(bs), 0, st, pl.subs, pl.bsubs, k, bwd, lca,
                       ybuf, bt, v, scale, nx, ny, s, s16);
    if (gemm_ev) (void)hipEventRecord(gemm_ev[2 * step], st);
    BlrStep<R, Z>::gemm(pl, k, bwd, astore, bt, ybuf, z, nx, ny, s, s16, st);
    if (gemm_ev) (void)hipEventRecord(gemm_ev[2 * step + 1], st);
  }
}

template void launch_blr_plane_max<float>(const SubDesc*, int, int, const float2*, double*,
                                          hipStream_t);
template void launch_blr_plane_max<double>(const SubDesc*, int, int, const double2*, double*,
                                           hipStream_t);
template void launch_blr_compress<float>(const SubDesc*, const BlrSub*, const BlrBlock*, long long,
                                         const float2*, const double*, int, double, int*, float2*,
                                         int*, hipStream_t);
template void launch_blr_compress<double>(const SubDesc*, const BlrSub*, const BlrBlock*, long long,
                                          const double2*, const double*, int, double, int*,
                                          double2*, int*, hipStream_t);
template void launch_oras_apply_blr<float, float2>(const BlrApply&, const float2*, const float2*,
                                                   float2*, float2*, const double2*, const double*,
                                                   float2*, int, int, int, hipStream_t,
                                                   hipEvent_t*);
template void launch_oras_apply_blr<float, double2>(const BlrApply&, const float2*, const float2*,
                                                    float2*, float2*, const double2*,
                                                    const double*, double2*, int, int, int,
                                                    hipStream_t, hipEvent_t*);
template void launch_oras_apply_blr<double, double2>(const BlrApply&, const double2*,
                                                     const double2*, double2*, double2*,
                                                     const double2*, const double*, double2*, int,
                                                     int, int, hipStream_t, hipEvent_t*);

}  // namespace oras
