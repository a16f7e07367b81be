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
//   * the right-hand side t is written into the subdomain's part of the
//     operand buffer in patch-major order (each patch's rows consecutive,
//     padded with zero rows to a multiple of 8);
//   * projection: for every column patch J, T_J = V_J t_J (V_J: the V of the
//     patch's low-rank blocks, stacked), each row stored with the rows that
//     its row patch I needs (T_I = [T_IJ for the low-rank J], consecutive);
//   * expansion: for every row patch I,
//         y_I = [S_II | S_IJ (dense blocks) | U_IJ (low-rank)] [t_I; t_J; T_I],
//     whose operand rows form a few runs of consecutive buffer rows; the
//     epilogue stores the plane rows and, on final planes, the owned nodes
//     (the same restricted prolongation as the dense substitution).
// Both are GEMMs on MFMA with the stored operand in [k / 4][row][k % 4]
// order and affine operand rows inside each run, so loads do not wait on
// other loads.  Compression runs twice: a first pass finds the ranks, the
// host lays out the operands, and a second pass (the same deterministic
// kernel) writes them.
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
// Operand-buffer row (from bt_off) of plane node (qx, qy): its patch's first
// t row plus its index inside the patch.  The patch along x is the part t
// with floor(t sx / npx) <= qx < floor((t+1) sx / npx), i.e.
// t = floor(((qx + 1) npx - 1) / sx); likewise along y.
__device__ inline int t_row(const SubDesc& sd, const BlrSub& bs, const int* __restrict__ lists,
                            int qx, int qy) {
  const int px = ((qx + 1) * bs.npx - 1) / sd.sx, py = ((qy + 1) * bs.npy - 1) / sd.sy;
  const int x0 = px * sd.sx / bs.npx, x1 = (px + 1) * sd.sx / bs.npx;
  const int y0 = py * sd.sy / bs.npy;
  return lists[bs.ptab + py * bs.npx + px] + (qy - y0) * (x1 - x0) + (qx - x0);
}

// Right-hand side entry t[q][c]: forward scale * v - L_k y_{k-1}, backward
// U_k x_{k+1} (couplings leaving the box are exact zeros in the local
// coefficients, so clamped neighbour indices contribute nothing).
template <typename R, int NC>
__device__ inline void rhs_entries(const SubDesc& sd, int k, int bwd, int qx, int qy, int c,
                                   const C<R>* __restrict__ lca, const C<R>* __restrict__ ybuf,
                                   const double2* __restrict__ v, const double* __restrict__ scale,
                                   int nx, int ny, int s, C<R>* t) {
  using T = C<R>;
#pragma unroll
  for (int j = 0; j < NC; ++j) t[j] = mk<R>(0, 0);
  if (!bwd) {
    const long long g = ((long long)(sd.lo[2] + k) * ny + sd.lo[1] + qy) * nx + sd.lo[0] + qx;
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      const double2 vv = v[g * s + c + j];
      const double sc = scale ? scale[c + j] : 1.0;
      t[j].x = (R)(vv.x * sc);
      t[j].y = (R)(vv.y * sc);
    }
  }
  if (bwd || k > 0) {
    const long long nbox = (long long)sd.sx * sd.sy * sd.sz;
    const long long node = ((long long)k * sd.sy + qy) * sd.sx + qx;
    const T* L = lca + sd.lca_off;
    const T* Yn = ybuf + (sd.y_off + (long long)(bwd ? k + 1 : k - 1) * sd.P) * s + c;
    const int ez = bwd ? 1 : -1;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
      const int py = min(max(qy + dy, 0), sd.sy - 1);
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int px = min(max(qx + dx, 0), sd.sx - 1);
        const T l = L[eidx(dx, dy, ez) * nbox + node];
        const T* yr = Yn + (long long)(py * sd.sx + px) * s;
#pragma unroll
        for (int j = 0; j < NC; ++j) {
          if (bwd) cfma(t[j], l, yr[j]);
          else cfms(t[j], l, yr[j]);
        }
      }
    }
  }
}

// FP32: sixteen lanes per plane row, two columns each (whole cache lines per
// load), one 16-byte store per lane.  The nine couplings of the block's rows
// to the neighbouring plane are staged in LDS once, not loaded by every lane
// of a row.
constexpr int RB_ROWS = 16;
__global__ void __launch_bounds__(RB_ROWS * 16)
blr_rhs_f32_kernel(const SubDesc* __restrict__ subs, const BlrSub* __restrict__ bsubs,
                   const int* __restrict__ lists, int nrb, int k, int bwd,
                   const float2* __restrict__ lca, const float2* __restrict__ ybuf,
                   float2* __restrict__ bt, const double2* __restrict__ v,
                   const double* __restrict__ scale, int nx, int ny, int s, int s16) {
  __shared__ float2 cpl[9][RB_ROWS];
  const SubDesc sd = subs[blockIdx.y];
  if (!plane_active(sd, k, bwd)) return;
  const int rb = blockIdx.x % nrb, cc = blockIdx.x / nrb;
  const bool couple = bwd || k > 0;
  if (couple) {
    const long long nbox = (long long)sd.sx * sd.sy * sd.sz;
    const int ez = bwd ? 1 : -1;
    const float sg = bwd ? 1.f : -1.f;
    for (int i = threadIdx.x; i < 9 * RB_ROWS; i += RB_ROWS * 16) {
      const int e = i / RB_ROWS, r = i % RB_ROWS, qq = rb * RB_ROWS + r;
      float2 l = make_float2(0.f, 0.f);
      if (qq < sd.p) {
        const long long node = ((long long)k * sd.sy + qq / sd.sx) * sd.sx + qq % sd.sx;
        l = lca[sd.lca_off + eidx(e % 3 - 1, e / 3 - 1, ez) * nbox + node];
        l.x *= sg;
        l.y *= sg;
      }
      cpl[e][r] = l;
    }
    __syncthreads();
  }
  const int rl = threadIdx.x >> 4;
  const int q = rb * RB_ROWS + rl;
  const int c = 32 * cc + 2 * (threadIdx.x & 15);
  if (q >= sd.p || c >= s) return;                 // s is even
  const int qx = q % sd.sx, qy = q / sd.sx;
  float2 t[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) t[j] = make_float2(0.f, 0.f);
  if (!bwd) {
    const long long g = ((long long)(sd.lo[2] + k) * ny + sd.lo[1] + qy) * nx + sd.lo[0] + qx;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const double2 vv = v[g * s + c + j];
      const double sc = scale ? scale[c + j] : 1.0;
      t[j] = make_float2((float)(vv.x * sc), (float)(vv.y * sc));
    }
  }
  if (couple) {
    const float2* Yn = ybuf + (sd.y_off + (long long)(bwd ? k + 1 : k - 1) * sd.P) * s + c;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
      const int py = min(max(qy + dy, 0), sd.sy - 1);
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int px = min(max(qx + dx, 0), sd.sx - 1);
        const float2 l = cpl[(dy + 1) * 3 + dx + 1][rl];
        const float4 yr = *reinterpret_cast<const float4*>(Yn + (long long)(py * sd.sx + px) * s);
        cfma(t[0], l, make_float2(yr.x, yr.y));
        cfma(t[1], l, make_float2(yr.z, yr.w));
      }
    }
  }
  const BlrSub bs = bsubs[blockIdx.y];
  *reinterpret_cast<float4*>(bt + (bs.bt_off + t_row(sd, bs, lists, qx, qy)) * s16 + c) =
      make_float4(t[0].x, t[0].y, t[1].x, t[1].y);
}

// FP64: one thread per entry.
__global__ void blr_rhs_f64_kernel(const SubDesc* __restrict__ subs,
                                   const BlrSub* __restrict__ bsubs, const int* __restrict__ lists,
                                   int k, int bwd, const double2* __restrict__ lca,
                                   const double2* __restrict__ ybuf, double2* __restrict__ bt,
                                   const double2* __restrict__ v, const double* __restrict__ scale,
                                   int nx, int ny, int s, int s16) {
  const SubDesc sd = subs[blockIdx.y];
  if (!plane_active(sd, k, bwd)) return;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)sd.p * s) return;
  const int q = (int)(idx / s), c = (int)(idx % s);
  const int qx = q % sd.sx, qy = q / sd.sx;
  double2 t[1];
  rhs_entries<double, 1>(sd, k, bwd, qx, qy, c, lca, ybuf, v, scale, nx, ny, s, t);
  const BlrSub bs = bsubs[blockIdx.y];
  bt[(bs.bt_off + t_row(sd, bs, lists, qx, qy)) * s16 + c] = t[0];
}

// --------------------------------------------------------- segment GEMMs --
// Work-group id -> (item, column group), with the items ordered so that every
// subdomain's items sit on one XCD.
__device__ inline bool item_map(int nitems, int ncg, int& it, int& cg) {
  const int b = blockIdx.x, r = b / NXCD;
  it = (r / ncg) * NXCD + b % NXCD;
  cg = r % ncg;
  return it < nitems;
}

// Complex FP32 on the bf16 instruction (32x32x16) with exactly split operands,
// as the dense plane products: every FP32 value of both operands is split
// into three bf16 pieces and six piece products form each real product, so
// each product carries an FP32-level error and accumulates in FP32.  One
// wave takes 32 rows and one 32-column chunk; the real and imaginary parts
// are separate accumulators.  A 16-k step covers four 4-row groups of the
// stored operand: lane (n = lane % 32, g = lane / 32) holds the operand
// entries (row n, k = 4 q + 2 g + e) and the t or T values (k = 4 q + 2 g + e,
// column n), value i = 2 q + e of both instruction operands referring to the
// same k.  A run of 4 m + 2 groups ends with a step whose last two groups are
// zeroed in the stored operand.
template <int MODE, typename Z>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2)))
blr_gemm_x3_kernel(const SubDesc* __restrict__ subs, const BlrSub* __restrict__ bsubs,
                   const BlrItem* __restrict__ items, int nitems, int ncg, int k, int bwd,
                   const float2* __restrict__ astore, const int* __restrict__ lists,
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
  const float2* btc = bt + bs.bt_off * s16;
  const float4* A = reinterpret_cast<const float4*>(astore + item.a_off);
  const int lane = threadIdx.x, n = lane & 31, g = lane >> 5;
  // columns at or beyond s16 read column s16 - 1 (in bounds; their results are dropped)
  const int colb = min(32 * cg + n, s16 - 1);
  f32x16 accR, accI;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    accR[j] = 0.f;
    accI[j] = 0.f;
  }
  // groups kq .. kq + 3 of the run [q0, q1) whose group q0 starts at
  // operand-buffer row rbase0; groups past the end repeat the last one with
  // the stored operand zeroed
  auto load = [&](int kq, int q0, int q1, int rbase0, float4 (&a)[4], float2 (&b)[8]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int gq = min(kq + q, q1 - 1);
      a[q] = A[((long long)gq * item.mpad + item.row0 + n) * 2 + g];
      if (kq + q >= q1) a[q] = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int e = 0; e < 2; ++e)
        b[2 * q + e] = btc[(long long)(rbase0 + 4 * (gq - q0) + 2 * g + e) * s16 + colb];
    }
  };
  auto mma = [&](const float4 (&a)[4], const float2 (&b)[8]) {
    unsigned r1[4], r2[4], r3[4], i1[4], i2[4], i3[4];
    unsigned s1[4], s2[4], s3[4], t1[4], t2[4], t3[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      split3(a[q].x, a[q].z, r1[q], r2[q], r3[q]);
      split3(a[q].y, a[q].w, i1[q], i2[q], i3[q]);
      split3(b[2 * q].x, b[2 * q + 1].x, s1[q], s2[q], s3[q]);
      split3(b[2 * q].y, b[2 * q + 1].y, t1[q], t2[q], t3[q]);
    }
    const u32x4 sgn = {0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
    const bf16x8 Ar1 = as_bf16x8(u32x4{r1[0], r1[1], r1[2], r1[3]});
    const bf16x8 Ar2 = as_bf16x8(u32x4{r2[0], r2[1], r2[2], r2[3]});
    const bf16x8 Ar3 = as_bf16x8(u32x4{r3[0], r3[1], r3[2], r3[3]});
    const bf16x8 Ai1 = as_bf16x8(u32x4{i1[0], i1[1], i1[2], i1[3]});
    const bf16x8 Ai2 = as_bf16x8(u32x4{i2[0], i2[1], i2[2], i2[3]});
    const bf16x8 Ai3 = as_bf16x8(u32x4{i3[0], i3[1], i3[2], i3[3]});
    const bf16x8 Ni1 = as_bf16x8(u32x4{i1[0], i1[1], i1[2], i1[3]} ^ sgn);
    const bf16x8 Ni2 = as_bf16x8(u32x4{i2[0], i2[1], i2[2], i2[3]} ^ sgn);
    const bf16x8 Ni3 = as_bf16x8(u32x4{i3[0], i3[1], i3[2], i3[3]} ^ sgn);
    const bf16x8 Br1 = as_bf16x8(u32x4{s1[0], s1[1], s1[2], s1[3]});
    const bf16x8 Br2 = as_bf16x8(u32x4{s2[0], s2[1], s2[2], s2[3]});
    const bf16x8 Br3 = as_bf16x8(u32x4{s3[0], s3[1], s3[2], s3[3]});
    const bf16x8 Bi1 = as_bf16x8(u32x4{t1[0], t1[1], t1[2], t1[3]});
    const bf16x8 Bi2 = as_bf16x8(u32x4{t2[0], t2[1], t2[2], t2[3]});
    const bf16x8 Bi3 = as_bf16x8(u32x4{t3[0], t3[1], t3[2], t3[3]});
#define ORAS_BX3(AR, AI, NI, BR, BI)                                           \
  accR = __builtin_amdgcn_mfma_f32_32x32x16_bf16(AR, BR, accR, 0, 0, 0);       \
  accI = __builtin_amdgcn_mfma_f32_32x32x16_bf16(AR, BI, accI, 0, 0, 0);       \
  accR = __builtin_amdgcn_mfma_f32_32x32x16_bf16(NI, BI, accR, 0, 0, 0);       \
  accI = __builtin_amdgcn_mfma_f32_32x32x16_bf16(AI, BR, accI, 0, 0, 0);
    ORAS_BX3(Ar1, Ai1, Ni1, Br1, Bi1)
    ORAS_BX3(Ar1, Ai1, Ni1, Br2, Bi2)
    ORAS_BX3(Ar2, Ai2, Ni2, Br1, Bi1)
    ORAS_BX3(Ar1, Ai1, Ni1, Br3, Bi3)
    ORAS_BX3(Ar3, Ai3, Ni3, Br1, Bi1)
    ORAS_BX3(Ar2, Ai2, Ni2, Br2, Bi2)
#undef ORAS_BX3
  };
  // one run of groups [q0, q1): the next 16-k step is fetched while the
  // current one feeds the products (loads past the end stay in bounds)
  auto run = [&](int q0, int q1, int rbase0) {
    float4 sa[4];
    float2 sb[8];
    load(q0, q0, q1, rbase0, sa, sb);
    for (int kq = q0; kq < q1; kq += 4) {
      float4 ca[4];
      float2 cb[8];
#pragma unroll
      for (int q = 0; q < 4; ++q) ca[q] = sa[q];
#pragma unroll
      for (int j = 0; j < 8; ++j) cb[j] = sb[j];
      load(kq + 4, q0, q1, rbase0, sa, sb);
      mma(ca, cb);
    }
  };
  if (MODE == 0) {
    run(0, item.K >> 2, item.brow);
  } else {
    for (int sg = 0; sg < item.nseg; ++sg) {
      const int4 seg = *reinterpret_cast<const int4*>(lists + item.list_off + 4 * sg);
      run(seg.x >> 2, (seg.x + seg.z) >> 2, seg.y);
    }
  }
  // accumulator item i of lane l: row 8 (i / 4) + 4 (l / 32) + i % 4, column l % 32
  const int col = 32 * cg + n;
  if (MODE == 0) {
    // destination rows first (all loads in flight together), then the stores
    int dest[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) dest[i] = lists[item.list_off + 8 * (i / 4) + 4 * g + (i % 4)];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int lr = 8 * (i / 4) + 4 * g + (i % 4);
      if (lr >= item.rows || col >= s) continue;
      bt[(bs.bt_off + dest[i]) * s16 + col] = make_float2(accR[i], accI[i]);
    }
    return;
  }
  int x0, w, y0, hh;
  patch_box(sd.sx, sd.sy, bs.npx, bs.npy, item.patch, x0, w, y0, hh);
  const int bsz = w * hh;
  const bool final_plane = bwd || (k == sd.sz - 1);
  float2* Yk = ybuf + (sd.y_off + (long long)k * sd.P) * s;
  const int colc = min(col, s - 1);
  // backward: x_k = y_k - (...): read every old value first (all loads in
  // flight together), then write
  float2 old[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) old[i] = make_float2(0.f, 0.f);
  if (bwd) {
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int l = min(item.row0 + 8 * (i / 4) + 4 * g + (i % 4), bsz - 1);
      old[i] = Yk[(long long)((y0 + l / w) * sd.sx + x0 + l % w) * s + colc];
    }
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int l = item.row0 + 8 * (i / 4) + 4 * g + (i % 4);
    if (l >= bsz || col >= s) continue;
    const int qx = x0 + l % w, qy = y0 + l / w;
    float2 val = make_float2(accR[i], accI[i]);
    if (bwd) val = make_float2(old[i].x - val.x, old[i].y - val.y);
    Yk[(long long)(qy * sd.sx + qx) * s + col] = val;
    if (final_plane) {
      const int gx = sd.lo[0] + qx, gy = sd.lo[1] + qy, gz = sd.lo[2] + k;
      if (gx >= sd.olo[0] && gx < sd.ohi[0] && gy >= sd.olo[1] && gy < sd.ohi[1] &&
          gz >= sd.olo[2] && gz < sd.ohi[2]) {
        ZR* zr = reinterpret_cast<ZR*>(z + (((long long)gz * ny + gy) * nx + gx) * s + col);
        zr[0] = (ZR)val.x;
        zr[1] = (ZR)val.y;
      }
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
                    const double2* __restrict__ astore, const int* __restrict__ lists,
                    double2* __restrict__ bt, double2* __restrict__ ybuf,
                    double2* __restrict__ z, int nx, int ny, int s, int s16) {
  int it, cg;
  if (!item_map(nitems, ncg, it, cg)) return;
  const BlrItem item = items[it];
  if (item.sub < 0) return;
  const SubDesc sd = subs[item.sub];
  if (!plane_active(sd, k, bwd)) return;
  const BlrSub bs = bsubs[item.sub];
  const double2* btc = bt + bs.bt_off * s16;
  const double2* A = astore + item.a_off;
  const int lane = threadIdx.x, m = lane & 15, kk = lane >> 4;
  const int bn = m >> 1;
  const bool im = (m & 1) != 0;
  const int c0 = 16 * cg;
  // columns at or beyond s16 read column s16 - 1 (in bounds; their results are dropped)
  int colc[2];
#pragma unroll
  for (int ns = 0; ns < 2; ++ns) colc[ns] = min(c0 + 8 * ns + bn, s16 - 1);
  f64x4 acc[RG][2];
#pragma unroll
  for (int rg = 0; rg < RG; ++rg)
#pragma unroll
    for (int ns = 0; ns < 2; ++ns) acc[rg][ns] = f64x4{0, 0, 0, 0};
  // one 4-row group: lane kk takes operand row 4 kq + kk
  auto load = [&](int kq, int rbase, double2 (&bv)[2], double2 (&a)[RG]) {
    const long long row = rbase + kk;
#pragma unroll
    for (int ns = 0; ns < 2; ++ns) bv[ns] = btc[row * s16 + colc[ns]];
#pragma unroll
    for (int rg = 0; rg < RG; ++rg)
      a[rg] = A[((long long)kq * item.mpad + item.row0 + 16 * rg + m) * 4 + kk];
  };
  auto mma = [&](const double2 (&bv)[2], const double2 (&a)[RG]) {
#pragma unroll
    for (int ns = 0; ns < 2; ++ns) {
      const double b1 = im ? bv[ns].y : bv[ns].x;
      const double b2 = im ? bv[ns].x : -bv[ns].y;
#pragma unroll
      for (int rg = 0; rg < RG; ++rg) {
        acc[rg][ns] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rg].x, b1, acc[rg][ns], 0, 0, 0);
        acc[rg][ns] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rg].y, b2, acc[rg][ns], 0, 0, 0);
      }
    }
  };
  // two groups in flight in two register sets, as in the FP32 kernel (runs
  // are multiples of 8 rows: an even number of groups; nothing conditional)
  auto run = [&](int q0, int q1, int rbase0) {
    double2 b0[2], b1[2], a0[RG], a1[RG];
    auto ld = [&](int kq, double2 (&bv)[2], double2 (&a)[RG]) {
      const int g = min(kq, q1 - 1);
      load(g, rbase0 + 4 * (g - q0), bv, a);
    };
    ld(q0, b0, a0);
    ld(q0 + 1, b1, a1);
    __builtin_amdgcn_sched_barrier(0);
    for (int kq = q0; kq < q1; kq += 2) {
      mma(b0, a0);
      __builtin_amdgcn_sched_barrier(0);
      ld(kq + 2, b0, a0);
      __builtin_amdgcn_sched_barrier(0);
      mma(b1, a1);
      __builtin_amdgcn_sched_barrier(0);
      ld(kq + 3, b1, a1);
      __builtin_amdgcn_sched_barrier(0);
    }
  };
  if (MODE == 0) {
    run(0, item.K >> 2, item.brow);
  } else {
    for (int sg = 0; sg < item.nseg; ++sg) {
      const int4 seg = *reinterpret_cast<const int4*>(lists + item.list_off + 4 * sg);
      run(seg.x >> 2, (seg.x + seg.z) >> 2, seg.y);
    }
  }
  if (MODE == 0) {
#pragma unroll
    for (int rg = 0; rg < RG; ++rg)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int lr = 16 * rg + kk + 4 * t;
        if (lr >= item.rows) continue;
        double* Tf = reinterpret_cast<double*>(bt + (bs.bt_off + lists[item.list_off + lr]) * s16);
#pragma unroll
        for (int ns = 0; ns < 2; ++ns) {
          const int col = c0 + 8 * ns + bn;
          if (col >= s) continue;
          Tf[2 * col + (im ? 1 : 0)] = acc[rg][ns][t];
        }
      }
    return;
  }
  int x0, w, y0, hh;
  patch_box(sd.sx, sd.sy, bs.npx, bs.npy, item.patch, x0, w, y0, hh);
  const int bsz = w * hh;
  const bool final_plane = bwd || (k == sd.sz - 1);
  double* Yk = reinterpret_cast<double*>(ybuf + (sd.y_off + (long long)k * sd.P) * s);
#pragma unroll
  for (int rg = 0; rg < RG; ++rg)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int l = item.row0 + 16 * rg + kk + 4 * t;
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
  static void run(const BlrApply& pl, int k, int bwd, const float2* astore, const float2* lca,
                  float2* bt, float2* ybuf, const double2* v, const double* scale, Z* z, int nx,
                  int ny, int s, int s16, hipStream_t st, hipEvent_t* ev) {
    const int nrb = (int)((pl.max_p + RB_ROWS - 1) / RB_ROWS);
    const int ncc = (s + 31) / 32;
    hipLaunchKernelGGL(blr_rhs_f32_kernel, dim3((unsigned)(nrb * ncc), (unsigned)pl.nsub),
                       dim3(RB_ROWS * 16), 0, st, pl.subs, pl.bsubs, pl.lists, nrb, k, bwd, lca,
                       ybuf, bt, v, scale, nx, ny, s, s16);
    if (ev) (void)hipEventRecord(ev[0], st);
    const int ncg = (s + 31) / 32;
    if (pl.p_count[k] > 0)
      hipLaunchKernelGGL((blr_gemm_x3_kernel<0, Z>), dim3((unsigned)(pl.p_count[k] * ncg)),
                         dim3(64), 0, st, pl.subs, pl.bsubs, pl.items + pl.p_first[k],
                         pl.p_count[k], ncg, k, bwd, astore, pl.lists, bt, ybuf, z, nx, ny, s,
                         s16);
    hipLaunchKernelGGL((blr_gemm_x3_kernel<1, Z>), dim3((unsigned)(pl.e_count[k] * ncg)),
                       dim3(64), 0, st, pl.subs, pl.bsubs, pl.items + pl.e_first[k],
                       pl.e_count[k], ncg, k, bwd, astore, pl.lists, bt, ybuf, z, nx, ny, s, s16);
    if (ev) (void)hipEventRecord(ev[1], st);
  }
};
template <> struct BlrStep<double, double2> {
  static void run(const BlrApply& pl, int k, int bwd, const double2* astore, const double2* lca,
                  double2* bt, double2* ybuf, const double2* v, const double* scale, double2* z,
                  int nx, int ny, int s, int s16, hipStream_t st, hipEvent_t* ev) {
    const int bs = 256;
    hipLaunchKernelGGL(blr_rhs_f64_kernel,
                       dim3((unsigned)((pl.max_p * s + bs - 1) / bs), (unsigned)pl.nsub), dim3(bs),
                       0, st, pl.subs, pl.bsubs, pl.lists, k, bwd, lca, ybuf, bt, v, scale, nx, ny,
                       s, s16);
    if (ev) (void)hipEventRecord(ev[0], st);
    const int ncg = (s + 15) / 16;
    if (pl.p_count[k] > 0)
      hipLaunchKernelGGL((blr_gemm_f64_kernel<2, 0>), dim3((unsigned)(pl.p_count[k] * ncg)),
                         dim3(64), 0, st, pl.subs, pl.bsubs, pl.items + pl.p_first[k],
                         pl.p_count[k], ncg, k, bwd, astore, pl.lists, bt, ybuf, z, nx, ny, s,
                         s16);
    hipLaunchKernelGGL((blr_gemm_f64_kernel<2, 1>), dim3((unsigned)(pl.e_count[k] * ncg)),
                       dim3(64), 0, st, pl.subs, pl.bsubs, pl.items + pl.e_first[k],
                       pl.e_count[k], ncg, k, bwd, astore, pl.lists, bt, ybuf, z, nx, ny, s, s16);
    if (ev) (void)hipEventRecord(ev[1], st);
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
  for (int step = 0; step < nsteps; ++step) {
    const int bwd = step >= pl.max_sz ? 1 : 0;
    const int k = bwd ? 2 * pl.max_sz - 2 - step : step;
    BlrStep<R, Z>::run(pl, k, bwd, astore, lca, bt, ybuf, v, scale, z, nx, ny, s, s16, st,
                       gemm_ev ? gemm_ev + 2 * step : nullptr);
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
