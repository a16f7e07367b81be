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
// pivot blocks of several tiles (no row exchanges; a zero or non-finite pivot
// is reported, and the smallest pivot relative to the plane's largest entry
// is recorded):
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
// U[c', c] couples node c' of plane k-1 to node c of plane k.  The couplings
// of the tile's 32 columns are staged in LDS once (every row of the tile uses
// them).
template <typename R>
__global__ void __launch_bounds__(256) schur_T_kernel(const SubDesc* subs, int k, const C<R>* fac,
                                                      C<R>* tbuf, const C<R>* lca) {
  using T = C<R>;
  __shared__ T ucol[9][TILE];
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
  for (int i = threadIdx.x; i < 9 * TILE; i += 256) {
    // coupling of column c to its neighbour (c - d) in plane k - 1, d = (dx, dy)
    const int d = i / TILE, c = J * TILE + i % TILE;
    const int dx = d % 3 - 1, dy = d / 3 - 1;
    T u = czero<T>();
    if (c < sd.p) {
      const int px = c % sd.sx - dx, py = c / sd.sx - dy;
      if (px >= 0 && px < sd.sx && py >= 0 && py < sd.sy)
        u = L[eidx(dx, dy, 1) * nbox + ((long long)(k - 1) * sd.sy + py) * sd.sx + px];
    }
    ucol[d][i % TILE] = u;
  }
  __syncthreads();
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
          const T s = Sinv[mat_off(a, py * sd.sx + px, nt)];
          cfma(acc, s, ucol[(dy + 1) * 3 + dx + 1][c4 * 4 + cl]);
        }
      }
    }
    Tm[tile_off(I, J, nt) + e] = acc;
  }
}

// S_k = D_k - L_k T  (just D_k on the first plane), identity on the pad.
// stats[2 (sub max_sz + k)] receives the bits of max |S_k|^2 (a non-negative
// double, so its bits order as the value).
// The couplings of the tile's 32 rows to plane k - 1 are staged in LDS once
// (every column of the tile uses them).
template <typename R>
__global__ void __launch_bounds__(256) build_S_kernel(const SubDesc* subs, int k, C<R>* fac,
                                                      const C<R>* tbuf, const C<R>* lca,
                                                      unsigned long long* stats, int max_sz) {
  using T = C<R>;
  __shared__ double red[256];
  __shared__ T lrow[9][TILE];
  const SubDesc sd = subs[blockIdx.z];
  if (k >= sd.sz) return;
  const int nt = sd.nt;
  const int I = blockIdx.y, J = blockIdx.x;
  if (I >= nt || J >= nt) return;
  double big = 0.0;
  const long long P2 = (long long)sd.P * sd.P;
  T* S = fac + sd.fac_off + (long long)k * P2;
  const T* Tm = tbuf + sd.t_off;
  const long long nbox = (long long)sd.sx * sd.sy * sd.sz;
  const T* L = lca + sd.lca_off;
  if (k > 0) {
    for (int i = threadIdx.x; i < 9 * TILE; i += 256) {
      const int e = i / TILE, b = I * TILE + i % TILE;
      T l = czero<T>();
      if (b < sd.p)
        l = L[eidx(e % 3 - 1, e / 3 - 1, -1) * nbox +
              ((long long)k * sd.sy + b / sd.sx) * sd.sx + b % sd.sx];
      lrow[e][i % TILE] = l;
    }
    __syncthreads();
  }
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
            const T t = Tm[mat_off(qy * sd.sx + qx, c, nt)];
            cfms(v, lrow[(ey + 1) * 3 + ex + 1][r], t);
          }
        }
      }
      big = fmax(big, (double)v.x * v.x + (double)v.y * v.y);
    }
    S[tile_off(I, J, nt) + e] = v;
  }
  red[threadIdx.x] = big;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0 && red[0] > 0.0)
    atomicMax(&stats[2 * ((long long)blockIdx.z * max_sz + k)],
              (unsigned long long)__double_as_longlong(red[0]));
}

// ------------------------------------------------------- blocked Gauss-Jordan
// Pivot blocks of NBT tiles (32 NBT rows); the last block of a plane may be
// narrower.  Every pass reads and writes the whole plane matrix once, so wide
// blocks cut the HBM traffic of the inversion; NBT is what fits the pivot
// block in LDS for the unblocked inversion (128 x 128 FP32, 64 x 64 FP64).
template <typename R> struct GjBlock;
template <> struct GjBlock<float> { static constexpr int NBT = 4, THREADS = 1024; };
template <> struct GjBlock<double> { static constexpr int NBT = 2, THREADS = 256; };

// A_kk <- A_kk^{-1} for the pivot block (nb tiles from tile kb0) by unblocked
// Gauss-Jordan.  The block lives in registers, a 4 x 4 sub-block per thread
// ((NB / 4)^2 threads); each pivot step publishes the pivot row and column
// through LDS, so a step costs two barriers.
// stats[2 (sub max_sz + k) + 1] receives the bits of max 1 / |pivot|^2.
template <typename R>
__global__ void __launch_bounds__(GjBlock<R>::THREADS)
gj_diag_kernel(const SubDesc* subs, int k, int kb0, C<R>* fac, int* status,
               unsigned long long* stats, int max_sz) {
  using T = C<R>;
  constexpr int NB = TILE * GjBlock<R>::NBT;
  constexpr int G = NB / 4;                  // thread grid edge
  static_assert(G * G == GjBlock<R>::THREADS, "one 4 x 4 block per thread");
  __shared__ T rowb[NB], colb[NB];
  __shared__ int bad;
  const SubDesc sd = subs[blockIdx.x];
  if (k >= sd.sz || kb0 >= sd.nt) return;
  const int nb = min(GjBlock<R>::NBT, sd.nt - kb0);
  const int nr = nb * TILE;
  T* base = fac + sd.fac_off + (long long)k * sd.P * sd.P;
  const int tr = threadIdx.x / G, tc = threadIdx.x % G;
  const int r0 = 4 * tr, c0 = 4 * tc;
  const bool live = r0 < nr && c0 < nr;
  // entries (r0 + i, c0 + j): tile (r / 32, c / 32), four columns contiguous
  T a[4][4];
  T* blk = base + tile_off(kb0 + r0 / TILE, kb0 + c0 / TILE, sd.nt);
  if (live) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) a[i][j] = blk[in_tile((r0 + i) % TILE, (c0 % TILE) + j)];
  }
  if (threadIdx.x == 0) bad = 0;
  R mag_min = INFINITY;    // smallest |pivot|^2 seen (thread 0)
  for (int piv = 0; piv < nr; ++piv) {
    const int pi = piv - r0, pj = piv - c0;
    if (live) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (pi == i) {
#pragma unroll
          for (int j = 0; j < 4; ++j) rowb[c0 + j] = a[i][j];
        }
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (pj == j) {
#pragma unroll
          for (int i = 0; i < 4; ++i) colb[r0 + i] = a[i][j];
        }
    }
    __syncthreads();
    const T p = rowb[piv];
    const R mag = p.x * p.x + p.y * p.y;
    const bool ok = isfinite(p.x) && isfinite(p.y) && mag > Tiny<R>::v;
    const R inv = (R)1 / (ok ? mag : (R)1);
    T ip;
    ip.x = p.x * inv;
    ip.y = -p.y * inv;
    if (!ok && threadIdx.x == 0) bad = 1;
    if (ok && threadIdx.x == 0 && piv < sd.p - TILE * kb0) mag_min = fmin(mag_min, mag);
    if (live) {
      // every entry as if off the pivot row and column (straight-line code),
      // then the pivot row and column rewritten from the published copies
      T rv[4], f[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) rv[j] = rowb[c0 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i) f[i] = cmul(colb[r0 + i], ip);   // A_r,piv / p
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) cfms(a[i][j], f[i], rv[j]);
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (pi == i) {
#pragma unroll
          for (int j = 0; j < 4; ++j) a[i][j] = cmul(rv[j], ip);       // A_piv,c / p
        }
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (pj == j) {
#pragma unroll
          for (int i = 0; i < 4; ++i) {                               // -A_r,piv / p
            a[i][j].x = pi == i ? ip.x : -f[i].x;
            a[i][j].y = pi == i ? ip.y : -f[i].y;
          }
        }
    }
    __syncthreads();
  }
  // largest 1 / |pivot|^2 over the block's pivots
  const double inv_min = mag_min < INFINITY ? 1.0 / (double)mag_min : 0.0;
  if (live) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) blk[in_tile((r0 + i) % TILE, (c0 % TILE) + j)] = a[i][j];
  }
  if (threadIdx.x == 0 && bad) status[blockIdx.x] = 1;
  if (threadIdx.x == 0 && inv_min > 0.0)
    atomicMax(&stats[2 * ((long long)blockIdx.x * max_sz + k) + 1],
              (unsigned long long)__double_as_longlong(inv_min));
}

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// One wave's 32 x 32 complex tile product on MFMA: acc += X Y with X and Y
// 32 x 32 tiles in the tile layout (global or LDS).  visit(row, col, part,
// value) walks the lane's share of the result.
template <typename R> struct TileMma;

// Complex FP32 on the bf16 instruction (32x32x16) with exactly split operands
// (three bf16 pieces per FP32 value, six piece products per real product:
// FP32-level error).  The real and imaginary parts of the result are separate
// accumulators, Re += Xr Yr - Xi Yi, Im += Xr Yi + Xi Yr.  Per 16-k half tile
// a lane (r = l % 32, g = l / 32) holds X entries (r, 4 q + 2 g + e) of the
// tile layout (four float4 loads, q = 0..3, e = 0..1) and the Y entries
// (4 q + 2 g + e, r) of column r, so value i = 2 q + e of both operands refers
// to the same k.
template <> struct TileMma<float> {
  f32x16 accR, accI;
  __device__ void zero() {
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      accR[j] = 0.f;
      accI[j] = 0.f;
    }
  }
  __device__ void mac(const float2* __restrict__ X, const float2* __restrict__ Y) {
    const int lane = threadIdx.x & 63, rr = lane & 31, g = lane >> 5;
    const float4* X4 = reinterpret_cast<const float4*>(X);
    const u32x4 sgn = {0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
#pragma unroll
    for (int hj = 0; hj < 2; ++hj) {
      float4 a[4];
      float2 y[8];
#pragma unroll
      for (int q = 0; q < 4; ++q) a[q] = X4[(4 * hj + q) * 64 + rr * 2 + g];
#pragma unroll
      for (int i = 0; i < 8; ++i) y[i] = Y[in_tile(16 * hj + 4 * (i >> 1) + 2 * g + (i & 1), rr)];
      unsigned r1[4], r2[4], r3[4], i1[4], i2[4], i3[4];
      unsigned s1[4], s2[4], s3[4], t1[4], t2[4], t3[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        split3(a[q].x, a[q].z, r1[q], r2[q], r3[q]);
        split3(a[q].y, a[q].w, i1[q], i2[q], i3[q]);
        split3(y[2 * q].x, y[2 * q + 1].x, s1[q], s2[q], s3[q]);
        split3(y[2 * q].y, y[2 * q + 1].y, t1[q], t2[q], t3[q]);
      }
      const bf16x8 Xr1 = as_bf16x8(u32x4{r1[0], r1[1], r1[2], r1[3]});
      const bf16x8 Xr2 = as_bf16x8(u32x4{r2[0], r2[1], r2[2], r2[3]});
      const bf16x8 Xr3 = as_bf16x8(u32x4{r3[0], r3[1], r3[2], r3[3]});
      const bf16x8 Xi1 = as_bf16x8(u32x4{i1[0], i1[1], i1[2], i1[3]});
      const bf16x8 Xi2 = as_bf16x8(u32x4{i2[0], i2[1], i2[2], i2[3]});
      const bf16x8 Xi3 = as_bf16x8(u32x4{i3[0], i3[1], i3[2], i3[3]});
      const bf16x8 Xn1 = as_bf16x8(u32x4{i1[0], i1[1], i1[2], i1[3]} ^ sgn);
      const bf16x8 Xn2 = as_bf16x8(u32x4{i2[0], i2[1], i2[2], i2[3]} ^ sgn);
      const bf16x8 Xn3 = as_bf16x8(u32x4{i3[0], i3[1], i3[2], i3[3]} ^ sgn);
      const bf16x8 Yr1 = as_bf16x8(u32x4{s1[0], s1[1], s1[2], s1[3]});
      const bf16x8 Yr2 = as_bf16x8(u32x4{s2[0], s2[1], s2[2], s2[3]});
      const bf16x8 Yr3 = as_bf16x8(u32x4{s3[0], s3[1], s3[2], s3[3]});
      const bf16x8 Yi1 = as_bf16x8(u32x4{t1[0], t1[1], t1[2], t1[3]});
      const bf16x8 Yi2 = as_bf16x8(u32x4{t2[0], t2[1], t2[2], t2[3]});
      const bf16x8 Yi3 = as_bf16x8(u32x4{t3[0], t3[1], t3[2], t3[3]});
#define ORAS_X3(XR, XI, XN, YR, YI)                                              \
  accR = __builtin_amdgcn_mfma_f32_32x32x16_bf16(XR, YR, accR, 0, 0, 0);         \
  accI = __builtin_amdgcn_mfma_f32_32x32x16_bf16(XR, YI, accI, 0, 0, 0);         \
  accR = __builtin_amdgcn_mfma_f32_32x32x16_bf16(XN, YI, accR, 0, 0, 0);         \
  accI = __builtin_amdgcn_mfma_f32_32x32x16_bf16(XI, YR, accI, 0, 0, 0);
      ORAS_X3(Xr1, Xi1, Xn1, Yr1, Yi1)
      ORAS_X3(Xr1, Xi1, Xn1, Yr2, Yi2)
      ORAS_X3(Xr2, Xi2, Xn2, Yr1, Yi1)
      ORAS_X3(Xr1, Xi1, Xn1, Yr3, Yi3)
      ORAS_X3(Xr3, Xi3, Xn3, Yr1, Yi1)
      ORAS_X3(Xr2, Xi2, Xn2, Yr2, Yi2)
#undef ORAS_X3
    }
  }
  // accumulator item i of lane l: row 8 (i / 4) + 4 (l / 32) + i % 4, column l % 32
  template <typename F> __device__ void visit(F f) const {
    const int lane = threadIdx.x & 63, rr = lane & 31, g = lane >> 5;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int row = 8 * (i / 4) + 4 * g + (i % 4);
      f(row, rr, 0, accR[i]);
      f(row, rr, 1, accI[i]);
    }
  }
};

// Complex FP64 on the 16x16x4 FP64 instruction (operands A[row = l % 16][k =
// l / 16], B[k = l / 16][col = l % 16]; result item t of lane l is row
// l / 16 + 4 t): two 16-row halves x four 8-column groups.
template <> struct TileMma<double> {
  f64x4 acc[2][4];
  __device__ void zero() {
#pragma unroll
    for (int rs = 0; rs < 2; ++rs)
#pragma unroll
      for (int ns = 0; ns < 4; ++ns) acc[rs][ns] = f64x4{0, 0, 0, 0};
  }
  __device__ void mac(const double2* __restrict__ X, const double2* __restrict__ Y) {
    const int lane = threadIdx.x & 63, m = lane & 15, kk = lane >> 4;
    const bool odd = (m & 1) != 0;
#pragma unroll 2
    for (int q = 0; q < 8; ++q) {
      const double2 a0 = X[(q * TILE + m) * 4 + kk];
      const double2 a1 = X[(q * TILE + 16 + m) * 4 + kk];
      const int kr = 4 * q + kk;
#pragma unroll
      for (int ns = 0; ns < 4; ++ns) {
        const double2 v = Y[in_tile(kr, 8 * ns + (m >> 1))];
        const double b1 = odd ? v.y : v.x, b2 = odd ? v.x : -v.y;
        acc[0][ns] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0.x, b1, acc[0][ns], 0, 0, 0);
        acc[0][ns] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0.y, b2, acc[0][ns], 0, 0, 0);
        acc[1][ns] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1.x, b1, acc[1][ns], 0, 0, 0);
        acc[1][ns] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1.y, b2, acc[1][ns], 0, 0, 0);
      }
    }
  }
  template <typename F> __device__ void visit(F f) const {
    const int lane = threadIdx.x & 63, m = lane & 15, kk = lane >> 4;
#pragma unroll
    for (int rs = 0; rs < 2; ++rs)
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int ns = 0; ns < 4; ++ns)
          f(rs * 16 + kk + 4 * t, 8 * ns + (m >> 1), m & 1, acc[rs][ns][t]);
  }
};

// component index of entry (row, col, part) of a tile
__device__ inline int comp_of(int row, int col, int part) { return 2 * in_tile(row, col) + part; }

// Copy one tile (1024 complex entries) into LDS with the wave's lanes.
template <typename T>
__device__ inline void tile_to_lds(const T* __restrict__ g, T* __restrict__ lds) {
  const int lane = threadIdx.x & 63;
#pragma unroll 4
  for (int i = 0; i < 1024 / 64; ++i) lds[i * 64 + lane] = g[i * 64 + lane];
}

// A_kJ <- A_kk^{-1} A_kJ for the pivot block (rows kb0 .. kb0 + nb - 1) and
// one tile column J outside it: one work-group of NBT waves per (J, subdomain),
// wave t producing tile (kb0 + t, J).  The nb input tiles of column J are
// overwritten, so they are staged in LDS first.
template <typename R>
__global__ void __launch_bounds__(64 * GjBlock<R>::NBT)
gj_rowpanel_kernel(const SubDesc* subs, int k, int kb0, C<R>* fac) {
  using T = C<R>;
  constexpr int NBT = GjBlock<R>::NBT;
  __shared__ __align__(16) T sY[NBT][1024];
  const SubDesc sd = subs[blockIdx.y];
  const int J = blockIdx.x;
  if (k >= sd.sz || kb0 >= sd.nt || J >= sd.nt) return;
  const int nb = min(NBT, sd.nt - kb0);
  if (J >= kb0 && J < kb0 + nb) return;
  T* base = fac + sd.fac_off + (long long)k * sd.P * sd.P;
  const int wv = threadIdx.x >> 6;
  if (wv < nb) tile_to_lds(base + tile_off(kb0 + wv, J, sd.nt), sY[wv]);
  __syncthreads();
  if (wv >= nb) return;
  TileMma<R> mm;
  mm.zero();
  for (int u = 0; u < nb; ++u) mm.mac(base + tile_off(kb0 + wv, kb0 + u, sd.nt), sY[u]);
  R* out = reinterpret_cast<R*>(base + tile_off(kb0 + wv, J, sd.nt));
  mm.visit([&](int row, int col, int part, R v) { out[comp_of(row, col, part)] = v; });
}

// A_Ik <- -A_Ik A_kk^{-1} for one tile row I outside the pivot block: one
// work-group of NBT waves per (I, subdomain), wave t producing tile (I, kb0 + t);
// the nb input tiles of row I are staged in LDS first.
template <typename R>
__global__ void __launch_bounds__(64 * GjBlock<R>::NBT)
gj_colpanel_kernel(const SubDesc* subs, int k, int kb0, C<R>* fac) {
  using T = C<R>;
  constexpr int NBT = GjBlock<R>::NBT;
  __shared__ __align__(16) T sX[NBT][1024];
  const SubDesc sd = subs[blockIdx.y];
  const int I = blockIdx.x;
  if (k >= sd.sz || kb0 >= sd.nt || I >= sd.nt) return;
  const int nb = min(NBT, sd.nt - kb0);
  if (I >= kb0 && I < kb0 + nb) return;
  T* base = fac + sd.fac_off + (long long)k * sd.P * sd.P;
  const int wv = threadIdx.x >> 6;
  if (wv < nb) tile_to_lds(base + tile_off(I, kb0 + wv, sd.nt), sX[wv]);
  __syncthreads();
  if (wv >= nb) return;
  TileMma<R> mm;
  mm.zero();
  for (int u = 0; u < nb; ++u) mm.mac(sX[u], base + tile_off(kb0 + u, kb0 + wv, sd.nt));
  R* out = reinterpret_cast<R*>(base + tile_off(I, kb0 + wv, sd.nt));
  mm.visit([&](int row, int col, int part, R v) { out[comp_of(row, col, part)] = -v; });
}

// A_IJ <- A_IJ - A_Ik A_kJ (I, J outside the pivot block): one wave per tile.
// For each pivot tile u the tile A_uJ is staged in LDS and A_Iu is read from
// memory directly as the row operand; the tile A_IJ is read after the
// products.  One 8 KB LDS tile and few live registers let five waves share a
// SIMD (with both operands staged and A_IJ held through the loop, two).
// Work-group ids are mapped so that all tiles of one subdomain run on the same
// XCD and read the pivot row and column panels from its L2.
constexpr int NXCD = 8;
template <typename R>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3)))
gj_update_kernel(const SubDesc* subs, int nsub, int max_nt, int k, int kb0, C<R>* fac) {
  using T = C<R>;
  __shared__ __align__(16) T sY[1024];
  const int bid = blockIdx.x, r = bid / NXCD, items = max_nt * max_nt;
  const int sub = (r / items) * NXCD + bid % NXCD, item = r % items;
  if (sub >= nsub) return;
  const SubDesc sd = subs[sub];
  const int I = item / max_nt, J = item % max_nt;
  if (k >= sd.sz || kb0 >= sd.nt || I >= sd.nt || J >= sd.nt) return;
  const int nb = min(GjBlock<R>::NBT, sd.nt - kb0);
  if ((I >= kb0 && I < kb0 + nb) || (J >= kb0 && J < kb0 + nb)) return;
  T* base = fac + sd.fac_off + (long long)k * sd.P * sd.P;
  R* Cr = reinterpret_cast<R*>(base + tile_off(I, J, sd.nt));
  TileMma<R> mm;
  mm.zero();
  for (int u = 0; u < nb; ++u) {
    tile_to_lds(base + tile_off(kb0 + u, J, sd.nt), sY);
    __syncthreads();
    mm.mac(base + tile_off(I, kb0 + u, sd.nt), sY);
    __syncthreads();
  }
  R cv[32];
  {
    int n = 0;
    mm.visit([&](int row, int col, int part, R) { cv[n++] = Cr[comp_of(row, col, part)]; });
  }
  int n = 0;
  mm.visit([&](int row, int col, int part, R v) {
    Cr[comp_of(row, col, part)] = cv[n] - v;
    ++n;
  });
}

}  // namespace

template <typename R>
void launch_factor_plane(const SubDesc* subs_dev, int nsub, int k, int max_nt, int max_sz,
                         C<R>* fac, C<R>* tbuf, const C<R>* lca, int* status,
                         unsigned long long* stats, hipStream_t st) {
  const dim3 g2(max_nt, max_nt, nsub);
  const int nsub8 = (nsub + NXCD - 1) / NXCD * NXCD;
  constexpr int NBT = GjBlock<R>::NBT;
  if (k > 0)
    hipLaunchKernelGGL((schur_T_kernel<R>), g2, dim3(256), 0, st, subs_dev, k, fac, tbuf, lca);
  hipLaunchKernelGGL((build_S_kernel<R>), g2, dim3(256), 0, st, subs_dev, k, fac, tbuf, lca, stats,
                     max_sz);
  for (int kb0 = 0; kb0 < max_nt; kb0 += NBT) {
    hipLaunchKernelGGL((gj_diag_kernel<R>), dim3(nsub), dim3(GjBlock<R>::THREADS), 0, st, subs_dev,
                       k, kb0, fac, status, stats, max_sz);
    hipLaunchKernelGGL((gj_rowpanel_kernel<R>), dim3(max_nt, nsub), dim3(64 * NBT), 0, st,
                       subs_dev, k, kb0, fac);
    hipLaunchKernelGGL((gj_update_kernel<R>), dim3((unsigned)(nsub8 * max_nt * max_nt)), dim3(64),
                       0, st, subs_dev, nsub, max_nt, k, kb0, fac);
    hipLaunchKernelGGL((gj_colpanel_kernel<R>), dim3(max_nt, nsub), dim3(64 * NBT), 0, st,
                       subs_dev, k, kb0, fac);
  }
}

template void launch_factor_plane<float>(const SubDesc*, int, int, int, int, float2*, float2*,
                                         const float2*, int*, unsigned long long*, hipStream_t);
template void launch_factor_plane<double>(const SubDesc*, int, int, int, int, double2*, double2*,
                                          const double2*, int*, unsigned long long*, hipStream_t);

}  // namespace oras
