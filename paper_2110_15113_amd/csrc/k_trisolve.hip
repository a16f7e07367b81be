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
//   * a GEMM kernel with one wave per (subdomain, 32-row tile, column group)
//     streams its rows of S_k^{-1} from HBM and t through L2 into MFMA.
// The GEMM epilogue stores the plane's rows and, once a plane is final,
// writes the owned nodes to the output (restricted prolongation with a
// Boolean partition of unity: each output entry is written once, no
// atomics).
//
// Complex products on real MFMA: with A = Ar + i Ai and B = Br + i Bi, the
// interleaved output columns (Re, Im) of C = A B come from two real products
// per k-slice, Ar * [Br | Bi] + Ai * [-Bi | Br].
//
// Complex FP32 (the mixed-precision path) uses the 32x32x2 instruction, which
// on gfx950 sustains its full rate from a single wave with four independent
// accumulators (the 16x16x4 form does not).  t is written by the
// right-hand-side kernel directly in the operand order of that instruction,
// so each wave fetches one 1 KB row of A and one 1 KB block of t per 4-deep
// k-slice pair with no lane duplication; the second real operand [-Bi | Br]
// is formed by swapping adjacent lanes (DPP).
//
// Complex FP64 uses the 16x16x4 FP64 instruction with t in row-major order.
//
// Work-groups are one wave.  The hardware hands consecutive work-group ids to
// the 8 XCDs in turn, so the linear id is mapped such that all waves of one
// subdomain land on the same XCD and share its L2 copy of t.
#include <algorithm>

#include "oras_internal.h"

namespace oras {

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int NXCD = 8;

template <typename Z> struct Comp;
template <> struct Comp<float2> { typedef float type; };
template <> struct Comp<double2> { typedef double type; };

// Work-group id -> (subdomain, item) with all items of one subdomain on one XCD.
__device__ inline void xcd_map(int items, int& sub, int& item) {
  const int b = blockIdx.x, r = b / NXCD;
  sub = (r / items) * NXCD + b % NXCD;
  item = r % items;
}

// A plane step does work for a subdomain on every forward plane, and on the
// backward planes from sz - 2 down to its lowest owned plane: only owned nodes
// are written out and the backward recursion runs downward, so the planes
// below the owned range feed nothing.
__device__ inline bool plane_active(const SubDesc& sd, int k, int bwd) {
  return bwd ? (k <= sd.sz - 2 && k >= sd.olo[2] - sd.lo[2]) : (k < sd.sz);
}

// Right-hand side of one plane row q, column c (q < p, c < s):
// forward scale * v - L_k y_{k-1} (the L part only for k > 0), backward U_k x_{k+1}.
template <typename R>
__device__ inline C<R> plane_rhs_entry(const SubDesc& sd, int k, int bwd, int q, int c,
                                       const C<R>* __restrict__ lca, const C<R>* __restrict__ ybuf,
                                       const double2* __restrict__ v,
                                       const double* __restrict__ scale, int nx, int ny, int s) {
  using T = C<R>;
  T t;
  t.x = 0;
  t.y = 0;
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
    // couplings that leave the box are stored as exact zeros in the local
    // coefficients (the restricted rows drop them), so clamped neighbour
    // indices contribute nothing and the loads need no branches
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
  return t;
}

// ------------------------------------------------------- complex FP32 path --
// t in operand order: per subdomain, per block cb of 16 columns, per group g
// of 8 plane rows, per lane (h = lane / 32, rr = lane % 32) one float4 whose
// component 2 p + e is part (rr & 1) of t[8 g + 4 p + 2 h + e][16 cb + rr / 2]
// (zero beyond the plane or beyond column s).
//
// A work-group forms t for 32 plane rows (four groups of 8) and 32 columns
// (two column blocks).  Eight lanes share a row, four columns each, so every
// vector load of y or v covers whole cache lines of one row and a coupling
// coefficient is one broadcast per row, loaded once per four columns (with
// sixteen lanes of two columns: 63.2 against 61.9 us per plane step on 160^3,
// 32 RHS); the tile is transposed through LDS and written out as whole float4
// operands, two per thread.
constexpr int RB_ROWS = 32;
constexpr int RB_THREADS = RB_ROWS * 8;

__global__ void __launch_bounds__(RB_THREADS)
plane_rhs_f32_kernel(const SubDesc* __restrict__ subs, int nsub, int nrb, int ncc, int k, int bwd,
                     const float2* __restrict__ lca, const float2* __restrict__ ybuf,
                     float4* __restrict__ tvm, const double2* __restrict__ v,
                     const double* __restrict__ scale, int nx, int ny, int s, int s16) {
  __shared__ float2 tile[RB_ROWS][33];
  int sub, item;
  xcd_map(nrb * ncc, sub, item);
  if (sub >= nsub) return;
  const SubDesc sd = subs[sub];
  if (!plane_active(sd, k, bwd)) return;
  const int G = sd.P / 8;
  const int cc = item / nrb, g0 = 4 * (item % nrb);
  if (g0 >= G) return;

  const int tid = threadIdx.x;
  const int rl = tid >> 3, cp = tid & 7;
  const int q = 8 * g0 + rl;
  const int c = 32 * cc + 4 * cp;
  float2 t[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) t[j] = make_float2(0.f, 0.f);
  if (q < sd.p && c < s) {
    const int qx = q % sd.sx, qy = q / sd.sx;
    if (!bwd) {
      const long long gn = ((long long)(sd.lo[2] + k) * ny + sd.lo[1] + qy) * nx + sd.lo[0] + qx;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const double2 vj = v[gn * s + c + j];
        const double sj = scale ? scale[c + j] : 1.0;
        t[j] = make_float2((float)(vj.x * sj), (float)(vj.y * sj));
      }
    }
    if (bwd || k > 0) {
      const long long nbox = (long long)sd.sx * sd.sy * sd.sz;
      const long long node = ((long long)k * sd.sy + qy) * sd.sx + qx;
      const float2* L = lca + sd.lca_off;
      const float2* Yn = ybuf + (sd.y_off + (long long)(bwd ? k + 1 : k - 1) * sd.P) * s + c;
      const int ez = bwd ? 1 : -1;
      const float sg = bwd ? 1.f : -1.f;
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy) {
        const int py = min(max(qy + dy, 0), sd.sy - 1);
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          const int px = min(max(qx + dx, 0), sd.sx - 1);
          float2 l = L[eidx(dx, dy, ez) * nbox + node];
          l.x *= sg;
          l.y *= sg;
          const float4* yp = reinterpret_cast<const float4*>(Yn + (long long)(py * sd.sx + px) * s);
          const float4 y0 = yp[0], y1 = yp[1];
          cfma(t[0], l, make_float2(y0.x, y0.y));
          cfma(t[1], l, make_float2(y0.z, y0.w));
          cfma(t[2], l, make_float2(y1.x, y1.y));
          cfma(t[3], l, make_float2(y1.z, y1.w));
        }
      }
    }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) tile[rl][4 * cp + j] = t[j];
  __syncthreads();
  // two float4 per thread: column block 2 cc + cbl, row group g0 + gl, lane
#pragma unroll
  for (int o = 0; o < 2; ++o) {
    const int idx = tid + RB_THREADS * o;
    const int cbl = idx >> 8, gl = (idx >> 6) & 3, lane = idx & 63;
    const int cb = 2 * cc + cbl;
    if (cb >= s16 / 16 || g0 + gl >= G) continue;
    const int h = lane >> 5, rr = lane & 31, ci = 16 * cbl + (rr >> 1);
    float val[4];
#pragma unroll
    for (int j4 = 0; j4 < 4; ++j4) {
      const float2 w = tile[8 * gl + 4 * (j4 >> 1) + 2 * h + (j4 & 1)][ci];
      val[j4] = (rr & 1) ? w.y : w.x;
    }
    tvm[sd.tv_off * s16 / 2 + ((long long)cb * G + g0 + gl) * 64 + lane] =
        make_float4(val[0], val[1], val[2], val[3]);
  }
}

// Y_k (=|-=) S_k^{-1} t for one 32-row tile and NB blocks of 16 columns (one
// wave).  A row of the factor tile layout holds, for each 4-k slice, rows
// r = lane % 32 with entries 2 h, 2 h + 1 (h = lane / 32) in one float4; the
// matching t operands come from the float4 of the operand-order layout.  The
// operands advance by half tiles of 16 k: the next half tile of both is
// prefetched into registers while the current one feeds 8 NB instructions.
// The half-tile buffers keep the wave within 168 registers, so three waves
// share a SIMD (whole 32-k tiles took 202 registers and allowed two).
// The factor rows are streamed once per launch: non-temporal loads keep them
// from evicting the t operand, which every row tile of a subdomain re-reads
// from L2 (400 -> 394 us per plane step on 160^3, 32 RHS).
typedef float f32x4nt __attribute__((ext_vector_type(4)));
__device__ inline float4 ld_nt(const float4* p) {
  const f32x4nt v = __builtin_nontemporal_load(reinterpret_cast<const f32x4nt*>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}

template <typename Z, int NB>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3)))
plane_gemm_f32_kernel(const SubDesc* __restrict__ subs, int nsub, int max_nt, int ncg, int cb0,
                      int k, int bwd, const float2* __restrict__ fac,
                      const float4* __restrict__ tvm, float2* __restrict__ ybuf,
                      Z* __restrict__ z, int nx, int ny, int s, int s16) {
  using ZR = typename Comp<Z>::type;
  int sub, item;
  xcd_map(max_nt * ncg, sub, item);
  if (sub >= nsub) return;
  const SubDesc sd = subs[sub];
  if (!plane_active(sd, k, bwd)) return;
  const int I = item / ncg, cg = item % ncg;
  const int nt = sd.nt;
  if (I >= nt) return;
  const int P = sd.P, G = P / 8;
  const int cbf = cb0 + cg * NB;   // first column block of this wave
  const float4* A4 = reinterpret_cast<const float4*>(fac + sd.fac_off + (long long)k * P * P) +
                     (long long)I * nt * 512;
  const float4* B4 = tvm + sd.tv_off * s16 / 2 + (long long)cbf * G * 64;
  const int lane = threadIdx.x, rr = lane & 31, h = lane >> 5;
  const int aoff = rr * 2 + h;
  const bool odd = (rr & 1) != 0;

  f32x16 acc[NB][2];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      acc[b][0][j] = 0.f;
      acc[b][1][j] = 0.f;
    }
  // half tiles of 16 k: 4 float4 of A and 2 x NB float4 of t per lane
  float4 sa[4], sb[2][NB];
#pragma unroll
  for (int q = 0; q < 4; ++q) sa[q] = ld_nt(&A4[q * 64 + aoff]);
#pragma unroll
  for (int gg = 0; gg < 2; ++gg)
#pragma unroll
    for (int b = 0; b < NB; ++b) sb[gg][b] = B4[((long long)b * G + gg) * 64 + lane];

  for (int HJ = 0; HJ < 2 * nt; ++HJ) {
    float4 ca[4], cbv[2][NB];
#pragma unroll
    for (int q = 0; q < 4; ++q) ca[q] = sa[q];
#pragma unroll
    for (int gg = 0; gg < 2; ++gg)
#pragma unroll
      for (int b = 0; b < NB; ++b) cbv[gg][b] = sb[gg][b];
    if (HJ + 1 < 2 * nt) {
      const int J1 = (HJ + 1) >> 1, h1 = (HJ + 1) & 1;
#pragma unroll
      for (int q = 0; q < 4; ++q) sa[q] = ld_nt(&A4[(long long)J1 * 512 + (4 * h1 + q) * 64 + aoff]);
#pragma unroll
      for (int gg = 0; gg < 2; ++gg)
#pragma unroll
        for (int b = 0; b < NB; ++b)
          sb[gg][b] = B4[((long long)b * G + 4 * J1 + 2 * h1 + gg) * 64 + lane];
    }
#pragma unroll
    for (int gg = 0; gg < 2; ++gg)
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        const float4 a = ca[2 * gg + p];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const float ar = e ? a.z : a.x, ai = e ? a.w : a.y;
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            const float4 bv = cbv[gg][b];
            const float b1 = p ? (e ? bv.w : bv.z) : (e ? bv.y : bv.x);
            const float sw = __int_as_float(__builtin_amdgcn_update_dpp(
                __float_as_int(b1), __float_as_int(b1), 0xB1, 0xF, 0xF, false));
            const float b2 = odd ? sw : -sw;
            acc[b][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, b1, acc[b][0], 0, 0, 0);
            acc[b][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai, b2, acc[b][1], 0, 0, 0);
          }
        }
      }
  }

  // accumulator item i of lane l: row 8 (i / 4) + 4 (l / 32) + i % 4, real column l % 32
  const bool final_plane = bwd || (k == sd.sz - 1);
  float* Yk = reinterpret_cast<float*>(ybuf + (sd.y_off + (long long)k * P) * s);
  // backward: read every old value first (all loads in flight together)
  float old[16][NB];
#pragma unroll
  for (int i = 0; i < 16; ++i)
#pragma unroll
    for (int b = 0; b < NB; ++b) old[i][b] = 0.f;
  if (bwd) {
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int row = I * TILE + 8 * (i / 4) + 4 * h + (i % 4);
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int col = min(16 * (cbf + b) + (rr >> 1), s - 1);
        old[i][b] = Yk[(long long)row * 2 * s + 2 * col + (rr & 1)];
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int row = I * TILE + 8 * (i / 4) + 4 * h + (i % 4);
    float* yr = Yk + (long long)row * 2 * s;
    long long zoff = -1;
    if (final_plane && row < sd.p) {
      const int qx = row % sd.sx, qy = row / sd.sx;
      const int gx = sd.lo[0] + qx, gy = sd.lo[1] + qy, gz = sd.lo[2] + k;
      if (gx >= sd.olo[0] && gx < sd.ohi[0] && gy >= sd.olo[1] && gy < sd.ohi[1] &&
          gz >= sd.olo[2] && gz < sd.ohi[2])
        zoff = (((long long)gz * ny + gy) * nx + gx) * s;
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int col = 16 * (cbf + b) + (rr >> 1);
      if (col >= s) continue;
      const int fi = 2 * col + (rr & 1);
      float val = acc[b][0][i] + acc[b][1][i];
      if (bwd) val = old[i][b] - val;
      yr[fi] = val;
      if (zoff >= 0) reinterpret_cast<ZR*>(z + zoff)[fi] = (ZR)val;
    }
  }
}

template <typename Z>
void gemm_f32_dispatch(const OrasPlan& pl, int k, int bwd, const float2* fac, const float4* tvm,
                       float2* ybuf, Z* z, int nx, int ny, int s, hipStream_t st) {
  const int s16 = (int)pad16(s);
  const int nblk = s16 / 16;
  const int nsub8 = (pl.nsub + NXCD - 1) / NXCD * NXCD;
  const int pairs = nblk / 2;
  if (pairs > 0)
    hipLaunchKernelGGL((plane_gemm_f32_kernel<Z, 2>), dim3((unsigned)(nsub8 * pl.max_nt * pairs)),
                       dim3(64), 0, st, pl.subs, pl.nsub, pl.max_nt, pairs, 0, k, bwd, fac, tvm,
                       ybuf, z, nx, ny, s, s16);
  if (nblk % 2)
    hipLaunchKernelGGL((plane_gemm_f32_kernel<Z, 1>), dim3((unsigned)(nsub8 * pl.max_nt)), dim3(64),
                       0, st, pl.subs, pl.nsub, pl.max_nt, 1, nblk - 1, k, bwd, fac, tvm, ybuf, z,
                       nx, ny, s, s16);
}

// ------------------------------------------------------- complex FP64 path --
// Both 16x16x4 FP64 operands: A[row = lane % 16][k = lane / 16],
// B[k = lane / 16][col = lane % 16]; result item t of lane l is row l / 16 + 4 t,
// column l % 16 (checked on gfx950).
__global__ void plane_rhs_f64_kernel(const SubDesc* __restrict__ subs, int k, int bwd,
                                     const double2* __restrict__ lca,
                                     const double2* __restrict__ ybuf, double2* __restrict__ tvbuf,
                                     const double2* __restrict__ v,
                                     const double* __restrict__ scale, int nx, int ny, int s) {
  const SubDesc sd = subs[blockIdx.y];
  if (!plane_active(sd, k, bwd)) return;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)sd.P * s) return;
  const int q = (int)(idx / s), c = (int)(idx % s);
  double2 t = make_double2(0.0, 0.0);
  if (q < sd.p) t = plane_rhs_entry<double>(sd, k, bwd, q, c, lca, ybuf, v, scale, nx, ny, s);
  tvbuf[sd.tv_off * (long long)pad16(s) + idx] = t;
}

// Y_k (=|-=) S_k^{-1} t for one 32-row tile and 8 NS columns (one wave); a
// 16-row x 8-column x 4-k step is two instructions (real and imaginary A).
// Column group cg of the launch starts at column c0base + 8 NS cg.
template <int NS>
__global__ void __launch_bounds__(64)
plane_gemm_f64_kernel(const SubDesc* __restrict__ subs, int nsub, int max_nt, int ncg, int k,
                      int bwd, const double2* __restrict__ fac, const double2* __restrict__ tvbuf,
                      double2* __restrict__ ybuf, double2* __restrict__ z, int nx, int ny, int s,
                      int c0base) {
  int sub, item;
  xcd_map(max_nt * ncg, sub, item);
  if (sub >= nsub) return;
  const SubDesc sd = subs[sub];
  if (!plane_active(sd, k, bwd)) return;
  const int nt = sd.nt;
  const int I = item / ncg, c0 = c0base + 8 * NS * (item % ncg);
  if (I >= nt) return;
  const int P = sd.P;
  const double2* A = fac + sd.fac_off + (long long)k * P * P + (long long)I * nt * (TILE * TILE);
  const double2* Bm = tvbuf + sd.tv_off * pad16(s) + c0;
  double2* Yk = ybuf + (sd.y_off + (long long)k * P) * s;
  const int lane = threadIdx.x;
  const int m = lane & 15, kk = lane >> 4;
  const int bn = m >> 1;
  const bool im = (m & 1) != 0;
  f64x4 acc[2][NS];
#pragma unroll
  for (int rs = 0; rs < 2; ++rs)
#pragma unroll
    for (int ns = 0; ns < NS; ++ns) acc[rs][ns] = f64x4{0, 0, 0, 0};
  for (int J = 0; J < nt; ++J) {
    const double2* tA = A + (long long)J * (TILE * TILE);
#pragma unroll 2
    for (int q = 0; q < 8; ++q) {
      const int kc = J * TILE + q * 4 + kk;
      const double2 a0 = tA[(q * TILE + m) * 4 + kk];
      const double2 a1 = tA[(q * TILE + 16 + m) * 4 + kk];
      const double2* brow = Bm + (long long)kc * s + bn;
#pragma unroll
      for (int ns = 0; ns < NS; ++ns) {
        const double2 bv = brow[ns * 8];
        const double b1 = im ? bv.y : bv.x;
        const double b2 = im ? bv.x : -bv.y;
        acc[0][ns] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0.x, b1, acc[0][ns], 0, 0, 0);
        acc[0][ns] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0.y, b2, acc[0][ns], 0, 0, 0);
        acc[1][ns] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1.x, b1, acc[1][ns], 0, 0, 0);
        acc[1][ns] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1.y, b2, acc[1][ns], 0, 0, 0);
      }
    }
  }
  const bool final_plane = bwd || (k == sd.sz - 1);
#pragma unroll
  for (int rs = 0; rs < 2; ++rs)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = I * TILE + rs * 16 + kk + 4 * i;
      double* yr = reinterpret_cast<double*>(Yk + (long long)row * s + c0);
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
        double val = acc[rs][ns][i];
        if (bwd) val = yr[idx] - val;
        yr[idx] = val;
        if (zoff >= 0) reinterpret_cast<double*>(z + zoff)[idx] = val;
      }
    }
}

// Columns in groups of 8, at most 4 groups per wave: the accumulators of 4
// keep a wave at 138 registers (three waves per SIMD; 8 groups took 265 and
// one wave, and re-reading the factors costs less than that).  Fewer groups
// per wave when a plane step would otherwise launch fewer than 2048 waves
// (few or small subdomains): every column group is a work-group of the same
// launch, and the groups of one row tile share its factor rows in L2.  (On
// 64 subdomains of 28^2-node planes and 32 RHS, 2 groups per wave took
// 14.6 ms per apply, 1 group 15.7 ms, 4 groups 19.1 ms.)  A remainder of
// groups goes to a second launch.
void gemm_f64_dispatch(const OrasPlan& pl, int k, int bwd, const double2* fac,
                       const double2* tvbuf, double2* ybuf, double2* z, int nx, int ny, int s,
                       hipStream_t st) {
  const int nsub8 = (pl.nsub + NXCD - 1) / NXCD * NXCD;
  const int groups = s / RHS_ALIGN;
  int ns = 4;
  while (ns > 1 && (long long)nsub8 * pl.max_nt * (groups / ns) < 2048) ns >>= 1;
  const int full = groups / ns, rem = groups % ns;
  auto launch = [&](int nsw, int ncg, int c0base) {
    const dim3 grid((unsigned)(nsub8 * pl.max_nt * ncg));
#define ORAS_GEMM(NS_)                                                                           \
  hipLaunchKernelGGL((plane_gemm_f64_kernel<NS_>), grid, dim3(64), 0, st, pl.subs, pl.nsub,     \
                     pl.max_nt, ncg, k, bwd, fac, tvbuf, ybuf, z, nx, ny, s, c0base)
    switch (nsw) {
      case 1: ORAS_GEMM(1); break;
      case 2: ORAS_GEMM(2); break;
      case 3: ORAS_GEMM(3); break;
      default: ORAS_GEMM(4); break;
    }
#undef ORAS_GEMM
  };
  if (full > 0) launch(ns, full, 0);
  if (rem > 0) launch(rem, 1, full * ns * RHS_ALIGN);
}

template <typename Z>
void plane_step_f32(const OrasPlan& pl, int k, int bwd, const float2* fac, const float2* lca,
                    float2* ybuf, float2* tvbuf, const double2* v, const double* scale, Z* z,
                    int nx, int ny, int s, hipStream_t st, hipEvent_t* ev) {
  const int s16 = (int)pad16(s);
  const int nrb = (int)((pl.max_p + RB_ROWS - 1) / RB_ROWS);   // 32-row blocks
  const int ncc = (s16 + 31) / 32;                               // 32-column chunks
  const int nsub8 = (pl.nsub + NXCD - 1) / NXCD * NXCD;
  hipLaunchKernelGGL(plane_rhs_f32_kernel, dim3((unsigned)(nsub8 * nrb * ncc)), dim3(RB_THREADS), 0,
                     st, pl.subs, pl.nsub, nrb, ncc, k, bwd, lca, ybuf,
                     reinterpret_cast<float4*>(tvbuf), v, scale, nx, ny, s, s16);
  if (ev) (void)hipEventRecord(ev[0], st);
  gemm_f32_dispatch<Z>(pl, k, bwd, fac, reinterpret_cast<const float4*>(tvbuf), ybuf, z, nx, ny,
                       s, st);
  if (ev) (void)hipEventRecord(ev[1], st);
}

void plane_step_f64(const OrasPlan& pl, int k, int bwd, const double2* fac, const double2* lca,
                    double2* ybuf, double2* tvbuf, const double2* v, const double* scale,
                    double2* z, int nx, int ny, int s, hipStream_t st, hipEvent_t* ev) {
  const int bs = 256;
  const dim3 grhs((unsigned)((pl.max_p * s + bs - 1) / bs), (unsigned)pl.nsub);
  hipLaunchKernelGGL(plane_rhs_f64_kernel, grhs, dim3(bs), 0, st, pl.subs, k, bwd, lca, ybuf,
                     tvbuf, v, scale, nx, ny, s);
  if (ev) (void)hipEventRecord(ev[0], st);
  gemm_f64_dispatch(pl, k, bwd, fac, tvbuf, ybuf, z, nx, ny, s, st);
  if (ev) (void)hipEventRecord(ev[1], st);
}

template <typename R, typename Z> struct Stepper;
template <typename Z> struct Stepper<float, Z> {
  static void run(const OrasPlan& pl, int k, int bwd, const float2* fac, const float2* lca,
                  float2* ybuf, float2* tvbuf, const double2* v, const double* scale, Z* z, int nx,
                  int ny, int s, hipStream_t st, hipEvent_t* ev) {
    plane_step_f32<Z>(pl, k, bwd, fac, lca, ybuf, tvbuf, v, scale, z, nx, ny, s, st, ev);
  }
};
template <> struct Stepper<double, double2> {
  static void run(const OrasPlan& pl, int k, int bwd, const double2* fac, const double2* lca,
                  double2* ybuf, double2* tvbuf, const double2* v, const double* scale,
                  double2* z, int nx, int ny, int s, hipStream_t st, hipEvent_t* ev) {
    plane_step_f64(pl, k, bwd, fac, lca, ybuf, tvbuf, v, scale, z, nx, ny, s, st, ev);
  }
};

}  // namespace

template <typename R, typename Z>
void launch_oras_apply(const OrasPlan& plan, const C<R>* fac, const C<R>* lca, C<R>* ybuf,
                       C<R>* tvbuf, const double2* v, const double* scale, Z* z, int nx, int ny,
                       int s, hipStream_t st, hipEvent_t* gemm_ev) {
  const int nsteps = 2 * plan.max_sz - 1;
  for (int step = 0; step < nsteps; ++step) {
    const bool bwd = step >= plan.max_sz;
    const int k = bwd ? 2 * plan.max_sz - 2 - step : step;
    Stepper<R, Z>::run(plan, k, bwd ? 1 : 0, fac, lca, ybuf, tvbuf, v, scale, z, nx, ny, s, st,
                       gemm_ev ? gemm_ev + 2 * step : nullptr);
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
