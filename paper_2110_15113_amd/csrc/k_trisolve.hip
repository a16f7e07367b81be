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
// Complex FP32 (the mixed-precision path) runs its products on the bf16
// matrix instruction with every FP32 operand split exactly into three bf16
// pieces (see the section below): the real and imaginary parts of the result
// accumulate separately, Re = Ar Br - Ai Bi and Im = Ar Bi + Ai Br, six piece
// products each, and the kernel streams S_k^{-1} at HBM speed.
//
// Complex FP64 uses the 16x16x4 FP64 instruction with t in row-major order;
// the interleaved output columns (Re, Im) of C = A B come from two real
// products per k-slice, Ar * [Br | Bi] + Ai * [-Bi | Br].
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

// The plane right-hand side: forward scale * v - L_k y_{k-1} (the L part only
// for k > 0), backward U_k x_{k+1}.  Couplings that leave the box are stored
// as exact zeros in the local coefficients (the restricted rows drop them),
// so clamped neighbour indices contribute nothing and the loads need no
// branches.
//
// The kernel of the complex FP32 path forms t for 32 plane rows and 32
// columns per work-group: eight lanes share a row, four columns each, so
// every vector load of y or v covers whole cache lines of one row; the
// block's couplings are staged in LDS once (with sixteen lanes of two
// columns: 63.2 against 61.9 us per plane step on 160^3, 32 RHS).
constexpr int RB_ROWS = 32;
constexpr int RB_THREADS = RB_ROWS * 8;

// The factor rows are streamed once per launch: non-temporal loads keep them
// from evicting the t operand, which every row tile of a subdomain re-reads
// from L2 (400 -> 394 us per plane step on 160^3, 32 RHS, with the FP32
// instruction).
typedef float f32x4nt __attribute__((ext_vector_type(4)));
__device__ inline float4 ld_nt(const float4* p) {
  const f32x4nt v = __builtin_nontemporal_load(reinterpret_cast<const f32x4nt*>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}

// ------------------------------------- complex FP32 on bf16 matrix cores --
// The FP32 products run on the bf16 MFMA (32x32x16), which has 16 times the
// dense FP32 MFMA rate on gfx950.  Every FP32 operand is split exactly into
// three bf16 pieces, x = x1 + x2 + x3 (each piece the round-to-nearest of what
// the previous ones leave; an FP32 significand of 24 bits leaves at most 8
// bits for the last piece, so the split loses nothing), and a real product
// a b is formed from the six piece products whose size is at least 2^-16 of
// a1 b1: a1 b1, a1 b2, a2 b1, a1 b3, a3 b1, a2 b2.  The three products left
// out are below 2^-24 |a b|, so each product carries an FP32-level error and
// the MFMA accumulates in FP32, as the FP32 instruction does.  The kernel then
// streams S_k^{-1} at HBM speed instead of waiting on the FP32 MFMA rate.
//
// t is kept already split by the right-hand-side kernel (it is re-read by
// every row tile of a subdomain), per subdomain, per chunk cc of 32 columns,
// per half tile hj of 16 plane rows, per piece pi (0..2: real part, 3..5:
// imaginary part), per lane (n = lane % 32 the column, g = lane / 32): one
// 16-byte group of eight bf16 values, value i being the piece of
// t[16 hj + 4 (i / 2) + 2 g + i % 2][32 cc + n].  That row order matches the
// factor rows a lane loads from the tile layout (lane (r, g): row r, entries
// 4 q + 2 g + e of the half tile for q = 0..3, e = 0..1), so value i of the A
// and B operands of the instruction refer to the same k.
// Right-hand side of 32 plane rows and one 32-column chunk, written as pieces.
// Eight lanes share a plane row, four columns each (one coupling load per four
// columns); the tile then goes through LDS and each thread writes the three
// pieces of one part of one lane's values.
__global__ void __launch_bounds__(RB_THREADS)
plane_rhs_x3_kernel(const SubDesc* __restrict__ subs, int nsub, int nrb, int ncc, int k, int bwd,
                    const float2* __restrict__ lca, const float2* __restrict__ ybuf,
                    u32x4* __restrict__ tp, const double2* __restrict__ v,
                    const double* __restrict__ scale, int nx, int ny, int s, int s32) {
  __shared__ float2 tile[RB_ROWS][33];
  __shared__ float2 cpl[9][RB_ROWS];   // the block rows' couplings to plane k -+ 1
  int sub, item;
  xcd_map(nrb * ncc, sub, item);
  if (sub >= nsub) return;
  const SubDesc sd = subs[sub];
  if (!plane_active(sd, k, bwd)) return;
  const int cc = item / nrb, q0 = RB_ROWS * (item % nrb);
  if (q0 >= sd.P) return;

  const int tid = threadIdx.x;
  const int rl = tid >> 3, cp = tid & 7;
  const int q = q0 + rl;
  const int c = 32 * cc + 4 * cp;
  const bool couple = bwd || k > 0;
  // each coupling is loaded once per block instead of once per column group
  if (couple) {
    const long long nbox = (long long)sd.sx * sd.sy * sd.sz;
    const int ez = bwd ? 1 : -1;
    const float sg = bwd ? 1.f : -1.f;
    for (int i = tid; i < 9 * RB_ROWS; i += RB_THREADS) {
      const int e = i / RB_ROWS, r = i % RB_ROWS, qq = q0 + r;
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
    if (couple) {
      const float2* Yn = ybuf + (sd.y_off + (long long)(bwd ? k + 1 : k - 1) * sd.P) * s + c;
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy) {
        const int py = min(max(qy + dy, 0), sd.sy - 1);
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          const int px = min(max(qx + dx, 0), sd.sx - 1);
          const float2 l = cpl[(dy + 1) * 3 + dx + 1][rl];
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
  // thread -> (half tile hl of the two, part, lane (n, g)); 8 values each
  const int hl = tid >> 7, part = (tid >> 6) & 1, lane = tid & 63;
  const int n = lane & 31, g = lane >> 5;
  float val[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const float2 w = tile[16 * hl + 4 * (i >> 1) + 2 * g + (i & 1)][n];
    val[i] = part ? w.y : w.x;
  }
  unsigned p1[4], p2[4], p3[4];
#pragma unroll
  for (int d = 0; d < 4; ++d) split3(val[2 * d], val[2 * d + 1], p1[d], p2[d], p3[d]);
  const int hj = q0 / 16 + hl;
  u32x4* out = tp + sd.tv_off * s32 * 3 / 4 +
               (((long long)cc * (sd.P / 16) + hj) * 6 + 3 * part) * 64 + lane;
  out[0] = u32x4{p1[0], p1[1], p1[2], p1[3]};
  out[64] = u32x4{p2[0], p2[1], p2[2], p2[3]};
  out[128] = u32x4{p3[0], p3[1], p3[2], p3[3]};
}

// Y_k (=|-=) S_k^{-1} t for RT 32-row tiles and one 32-column chunk (one
// wave), on the bf16 instruction with split operands.  The real and imaginary
// parts of the result are separate accumulators:
//   Re += Ar Br - Ai Bi,  Im += Ar Bi + Ai Br,
// six piece products each, 24 instructions per 16 k and row tile; the RT row
// tiles share every t piece the wave loads.  The next half tile of the factor
// rows and of the t pieces is fetched while the current one feeds the
// products; the factor rows are streamed once (non-temporal loads).
template <typename Z, int RT>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(RT == 1 ? 3 : 2)))
plane_gemm_x3_kernel(const SubDesc* __restrict__ subs, int nsub, int max_ng, int ncc, int k,
                     int bwd, const float2* __restrict__ fac, const u32x4* __restrict__ tp,
                     float2* __restrict__ ybuf, Z* __restrict__ z, int nx, int ny, int s,
                     int s32) {
  using ZR = typename Comp<Z>::type;
  int sub, item;
  xcd_map(max_ng * ncc, sub, item);
  if (sub >= nsub) return;
  const SubDesc sd = subs[sub];
  if (!plane_active(sd, k, bwd)) return;
  const int I0 = (item / ncc) * RT, cc = item % ncc;
  const int nt = sd.nt;
  if (I0 >= nt) return;
  const int P = sd.P;
  const float4* A4[RT];
#pragma unroll
  for (int t = 0; t < RT; ++t)   // a tile beyond the plane repeats the last one, unstored
    A4[t] = reinterpret_cast<const float4*>(fac + sd.fac_off + (long long)k * P * P) +
            (long long)min(I0 + t, nt - 1) * nt * 512;
  const u32x4* B = tp + sd.tv_off * s32 * 3 / 4 + (long long)cc * (P / 16) * 6 * 64;
  const int lane = threadIdx.x, rr = lane & 31, g = lane >> 5;
  const int aoff = rr * 2 + g;

  f32x16 accR[RT], accI[RT];
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      accR[t][j] = 0.f;
      accI[t][j] = 0.f;
    }
  float4 sa[RT][4];
  u32x4 sb[6];
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) sa[t][q] = ld_nt(&A4[t][q * 64 + aoff]);
#pragma unroll
  for (int pi = 0; pi < 6; ++pi) sb[pi] = B[pi * 64 + lane];

  for (int HJ = 0; HJ < 2 * nt; ++HJ) {
    float4 ca[RT][4];
    u32x4 cb[6];
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) ca[t][q] = sa[t][q];
#pragma unroll
    for (int pi = 0; pi < 6; ++pi) cb[pi] = sb[pi];
    if (HJ + 1 < 2 * nt) {
      const int J1 = (HJ + 1) >> 1, h1 = (HJ + 1) & 1;
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          sa[t][q] = ld_nt(&A4[t][(long long)J1 * 512 + (4 * h1 + q) * 64 + aoff]);
#pragma unroll
      for (int pi = 0; pi < 6; ++pi) sb[pi] = B[((long long)(HJ + 1) * 6 + pi) * 64 + lane];
    }
    const bf16x8 Br1 = as_bf16x8(cb[0]), Br2 = as_bf16x8(cb[1]), Br3 = as_bf16x8(cb[2]);
    const bf16x8 Bi1 = as_bf16x8(cb[3]), Bi2 = as_bf16x8(cb[4]), Bi3 = as_bf16x8(cb[5]);
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      // value i = 2 q + e of the lane: real / imaginary part of entry e of ca[t][q]
      unsigned r1[4], r2[4], r3[4], i1[4], i2[4], i3[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        split3(ca[t][q].x, ca[t][q].z, r1[q], r2[q], r3[q]);
        split3(ca[t][q].y, ca[t][q].w, i1[q], i2[q], i3[q]);
      }
      const bf16x8 Ar1 = as_bf16x8(u32x4{r1[0], r1[1], r1[2], r1[3]});
      const bf16x8 Ar2 = as_bf16x8(u32x4{r2[0], r2[1], r2[2], r2[3]});
      const bf16x8 Ar3 = as_bf16x8(u32x4{r3[0], r3[1], r3[2], r3[3]});
      const bf16x8 Ai1 = as_bf16x8(u32x4{i1[0], i1[1], i1[2], i1[3]});
      const bf16x8 Ai2 = as_bf16x8(u32x4{i2[0], i2[1], i2[2], i2[3]});
      const bf16x8 Ai3 = as_bf16x8(u32x4{i3[0], i3[1], i3[2], i3[3]});
      const u32x4 sgn = {0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
      const bf16x8 Ni1 = as_bf16x8(u32x4{i1[0], i1[1], i1[2], i1[3]} ^ sgn);
      const bf16x8 Ni2 = as_bf16x8(u32x4{i2[0], i2[1], i2[2], i2[3]} ^ sgn);
      const bf16x8 Ni3 = as_bf16x8(u32x4{i3[0], i3[1], i3[2], i3[3]} ^ sgn);
#define ORAS_X3(AR, AI, NI, BR, BI)                                                \
  accR[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(AR, BR, accR[t], 0, 0, 0);     \
  accI[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(AR, BI, accI[t], 0, 0, 0);     \
  accR[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(NI, BI, accR[t], 0, 0, 0);     \
  accI[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(AI, BR, accI[t], 0, 0, 0);
      ORAS_X3(Ar1, Ai1, Ni1, Br1, Bi1)
      ORAS_X3(Ar1, Ai1, Ni1, Br2, Bi2)
      ORAS_X3(Ar2, Ai2, Ni2, Br1, Bi1)
      ORAS_X3(Ar1, Ai1, Ni1, Br3, Bi3)
      ORAS_X3(Ar3, Ai3, Ni3, Br1, Bi1)
      ORAS_X3(Ar2, Ai2, Ni2, Br2, Bi2)
#undef ORAS_X3
    }
  }

  // accumulator item i of lane l: row 8 (i / 4) + 4 (l / 32) + i % 4, column l % 32
  const bool final_plane = bwd || (k == sd.sz - 1);
  const int col = 32 * cc + rr;
  float2* Yk = ybuf + (sd.y_off + (long long)k * P) * s;
  const int colc = min(col, s - 1);
#pragma unroll
  for (int t = 0; t < RT; ++t) {
    const int I = I0 + t;
    if (I >= nt) break;
    // backward: read every old value first (all loads in flight together)
    float2 old[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) old[i] = make_float2(0.f, 0.f);
    if (bwd) {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int row = I * TILE + 8 * (i / 4) + 4 * g + (i % 4);
        old[i] = Yk[(long long)row * s + colc];
      }
    }
    if (col >= s) continue;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int row = I * TILE + 8 * (i / 4) + 4 * g + (i % 4);
      float2 val = make_float2(accR[t][i], accI[t][i]);
      if (bwd) val = make_float2(old[i].x - val.x, old[i].y - val.y);
      Yk[(long long)row * s + col] = val;
      if (final_plane && row < sd.p) {
        const int qx = row % sd.sx, qy = row / sd.sx;
        const int gx = sd.lo[0] + qx, gy = sd.lo[1] + qy, gz = sd.lo[2] + k;
        if (gx >= sd.olo[0] && gx < sd.ohi[0] && gy >= sd.olo[1] && gy < sd.ohi[1] &&
            gz >= sd.olo[2] && gz < sd.ohi[2]) {
          ZR* zp = reinterpret_cast<ZR*>(z + (((long long)gz * ny + gy) * nx + gx) * s + col);
          zp[0] = (ZR)val.x;
          zp[1] = (ZR)val.y;
        }
      }
    }
  }
}

// ------------------------------------------------------- complex FP64 path --
// Both 16x16x4 FP64 operands: A[row = lane % 16][k = lane / 16],
// B[k = lane / 16][col = lane % 16]; result item t of lane l is row l / 16 + 4 t,
// column l % 16 (checked on gfx950).

// The FP64 right-hand side, one thread per entry; the rows a 256-thread
// block touches (256 entries, s >= 8 of them per row, the first row possibly
// partial) have their couplings staged in LDS once.
constexpr int RHS64_ROWS = 256 / 8 + 1;
__global__ void __launch_bounds__(256)
plane_rhs_f64_kernel(const SubDesc* __restrict__ subs, int k, int bwd,
                                     const double2* __restrict__ lca,
                                     const double2* __restrict__ ybuf, double2* __restrict__ tvbuf,
                                     const double2* __restrict__ v,
                                     const double* __restrict__ scale, int nx, int ny, int s) {
  // the couplings of the block's rows (at most 256 / 8 + 1 of them) are
  // staged in LDS once, not loaded for every right-hand side
  __shared__ double2 cpl[9][RHS64_ROWS];
  const SubDesc sd = subs[blockIdx.y];
  if (!plane_active(sd, k, bwd)) return;
  const long long idx0 = (long long)blockIdx.x * blockDim.x;
  const long long idx = idx0 + threadIdx.x;
  const int qf = (int)(idx0 / s);
  const bool couple = bwd || k > 0;
  if (couple) {
    const long long nbox = (long long)sd.sx * sd.sy * sd.sz;
    const int ez = bwd ? 1 : -1;
    const double sg = bwd ? 1.0 : -1.0;
    for (int i = threadIdx.x; i < 9 * RHS64_ROWS; i += blockDim.x) {
      const int e = i / RHS64_ROWS, r = i % RHS64_ROWS, qq = qf + r;
      double2 l = make_double2(0.0, 0.0);
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
  if (idx >= (long long)sd.P * s) return;
  const int q = (int)(idx / s), c = (int)(idx % s);
  double2 t = make_double2(0.0, 0.0);
  if (q < sd.p) {
    const int qx = q % sd.sx, qy = q / sd.sx;
    if (!bwd) {
      const long long g = ((long long)(sd.lo[2] + k) * ny + sd.lo[1] + qy) * nx + sd.lo[0] + qx;
      const double2 vv = v[g * s + c];
      const double sc = scale ? scale[c] : 1.0;
      t = make_double2(vv.x * sc, vv.y * sc);
    }
    if (couple) {
      const double2* Yn = ybuf + (sd.y_off + (long long)(bwd ? k + 1 : k - 1) * sd.P) * s + c;
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy) {
        const int py = min(max(qy + dy, 0), sd.sy - 1);
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          const int px = min(max(qx + dx, 0), sd.sx - 1);
          cfma(t, cpl[(dy + 1) * 3 + dx + 1][q - qf], Yn[(long long)(py * sd.sx + px) * s]);
        }
      }
    }
  }
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
  const int s32 = (int)pad32(s);
  const int nrb = (int)((pl.max_p + RB_ROWS - 1) / RB_ROWS);   // 32-row blocks
  const int ncc = s32 / 32;                                      // 32-column chunks
  const int nsub8 = (pl.nsub + NXCD - 1) / NXCD * NXCD;
  u32x4* tp = reinterpret_cast<u32x4*>(tvbuf);
  hipLaunchKernelGGL(plane_rhs_x3_kernel, dim3((unsigned)(nsub8 * nrb * ncc)), dim3(RB_THREADS), 0,
                     st, pl.subs, pl.nsub, nrb, ncc, k, bwd, lca, ybuf, tp, v, scale, nx, ny, s,
                     s32);
  if (ev) (void)hipEventRecord(ev[0], st);
  // two row tiles per wave share each t piece they load: 278.8 -> 265.6 us
  // per plane step on 160^3, 32 RHS (212 registers, two waves per SIMD)
  constexpr int RT = 2;
  const int max_ng = (pl.max_nt + RT - 1) / RT;
  hipLaunchKernelGGL((plane_gemm_x3_kernel<Z, RT>), dim3((unsigned)(nsub8 * max_ng * ncc)),
                     dim3(64), 0, st, pl.subs, pl.nsub, max_ng, ncc, k, bwd, fac, tp, ybuf, z, nx,
                     ny, s, s32);
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
