// Matrix-free multi-RHS 27-point apply y = A x (or the residual y = b - A x).
//
// Paper sec. 2.3: A is the compact 27-point stencil whose stiffness and
// consistent-mass parts mix rotated coordinate systems, with weights picked
// per node from G.  Each row's coefficients are formed inside the kernel from
// node fields instead of being read from a stored array.
//
// Stiffness.  Three symmetric flux families: axis differences at face
// midpoints (weight W1), 2 x 2-averaged differences at in-plane cell centres
// (W2) and 2 x 2 x 2-averaged differences at cube centres (W3), the family
// weights (with their averaging factors and 1 / h^2) being the same for every
// G.  A staggered point at i + q/2 (q_a in {-1, +1} on its gradient axes)
// carries W_a = W K_a for each gradient axis a, K_a = S / s_a^2 the
// stretched-coordinate metric of the 1D PML profiles s_a (S = s_x s_y s_z at
// the point), so K_a is 1 / s_a at the point's half coordinate along a times
// s_b at its coordinate along every other axis b.  A point adds W_a to the
// coupling of each of its support nodes that moved along a and subtracts it
// from those that did not.  Summing over the points whose support holds both
// i and i + e, the coupling to offset e factorises per axis:
//   cube:      W3 sum_a sg_a R_a prod_{b != a} H_b
//   in-plane:  W2 N_c (sg_a R_a H_b + sg_b R_b H_a)   (plane ab, if e_c = 0)
//   axis:      W1 sg_a R_a N_b N_c                    (axis a, if e_b = e_c = 0)
// with sg_a = +1 if e_a != 0 and -1 otherwise, and per axis (offset d = e_a):
// R(+-1) = 1 / s(i +- 1/2), R(0) = R(-1) + R(+1); H likewise with s itself;
// N_b = s(i) on axis b.  These per-axis factors are tabulated per node
// coordinate on the host.  Where the PML does not reach a tile (every profile
// value its nodes use is 1) the stiffness is one value per shell and S = 1;
// such tiles run a kernel without the factor arithmetic.
//
// Mass.  mu_ii = omega^2 wm0_i m~_i S_i; for a neighbour j in shell t,
// mu_ij = omega^2 (wm_t,i + wm_t,j)/2 (m~_i + m~_j)/2 (S_i + S_j)/2.
//
// Tiling.  A work-group owns a TX x TY tile and a chunk of RC right-hand
// sides (up to 32 on PML tiles, 16 elsewhere in single precision) and
// streams the planes p = k0 - 1 .. k0 + TZ through LDS one at a time: each
// x value of plane p is read once from LDS and applied to the three outputs
// it couples to (planes p - 1, p and p + 1 of the same column), which the
// threads keep in registers and write once complete.  Four lanes (a DPP quad) share a node, RC / 4
// right-hand sides each: for every neighbour column, lane o forms the
// coupling of output plane p - 1 + o (lane 3 idles) and the quad exchanges
// the three couplings by DPP broadcasts, so a coupling is formed once per
// node and plane whatever the number of right-hand sides.  Node fields sit in
// a three-plane LDS ring; the next plane is fetched into registers while the
// current one is applied.  Ghost nodes outside the grid hold x = 0
// (Dirichlet), so their couplings need no special case.  Work items (tile,
// chunk) are dealt to the XCDs in contiguous ranges, so neighbouring tiles,
// which share halo columns, run on the same L2 at about the same time.
#include "oras_internal.h"

#include <algorithm>
#include <type_traits>
#include <utility>
#include <vector>

namespace oras {

namespace {

// Tiles of TX x TY x TZ nodes (measured on a 160^3 grid with 32 right-hand
// sides: 8 x 8 columns beat 16 x 8 and 16 x 4 by 2-6 %; marching 32 planes
// was no faster per node)
constexpr int TX = 8;
constexpr int TY = 8;
constexpr int TZ = 16;
constexpr int NXCD = 8;
constexpr int NS = 4;                  // lanes per node: one DPP quad
constexpr int NTHREADS = TX * TY * NS;

// widest chunk of right-hand sides per work-group.  PML tiles take 256 bytes
// per node (their couplings cost more arithmetic, formed once per chunk);
// PML-free tiles in single precision take 16 right-hand sides, which leaves
// room for two work-groups per CU.
template <typename R, bool PML> struct MfChunk;
template <bool PML> struct MfChunk<float, PML> { static constexpr int RC = PML ? 32 : 16; };
template <bool PML> struct MfChunk<double, PML> { static constexpr int RC = 16; };

template <typename R> __device__ inline C<R> cz() { C<R> z; z.x = 0; z.y = 0; return z; }
template <typename R> __device__ inline C<R> csc(C<R> a, R s) { a.x *= s; a.y *= s; return a; }

// An empty register constraint: the value must exist here, so the compiler
// can neither sink its computation past this point nor merge it with later
// uses.
template <typename T> __device__ inline void pin(T& v) {
  asm volatile("" : "+v"(v.x), "+v"(v.y));
}

// lane J's value of a quad, broadcast to its four lanes (DPP quad_perm)
template <int J> __device__ inline float quad_bcast(float v) {
  return __int_as_float(
      __builtin_amdgcn_mov_dpp(__float_as_int(v), J * 0x55, 0xf, 0xf, false));
}
template <int J> __device__ inline double quad_bcast(double v) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(u & 0xffffffffLL), J * 0x55, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(u >> 32), J * 0x55, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int J, typename T> __device__ inline T quad_bcast_c(T v) {
  v.x = quad_bcast<J>(v.x);
  v.y = quad_bcast<J>(v.y);
  return v;
}

// factor slots per node coordinate: R(d), H(d), N(d) for d = -1, 0, +1
__device__ inline constexpr int FR(int d) { return d + 1; }
__device__ inline constexpr int FH(int d) { return 4 + d; }
__device__ inline constexpr int FN(int d) { return 7 + d; }

template <int... I, typename F>
__device__ inline void static_for_impl(std::integer_sequence<int, I...>, F&& f) {
  (f(std::integral_constant<int, I>()), ...);
}
// f(integral_constant<int, i>) for i = 0 .. N - 1, unrolled at compile time
template <int N, typename F> __device__ inline void static_for(F&& f) {
  static_for_impl(std::make_integer_sequence<int, N>(), f);
}

// which outputs a plane step feeds: the plane before the tile only the
// tile's first plane, the plane after it only the last one
enum { FIRST = 0, MID = 1, LAST = 2 };

// PML: tiles the PML reaches (profile factors formed), else PML-free tiles.
// RC: right-hand sides of the work-group's chunk (a multiple of 8).
template <typename R, bool PML, int RC, typename Y>
__global__ void __launch_bounds__(NTHREADS)
stencil_mf_kernel(StencilMF<R> op, const int4* __restrict__ tiles, const C<R>* __restrict__ x,
                  const double2* __restrict__ b, Y* __restrict__ y, int nx, int ny, int nz,
                  int s, int c_first, int nitems, int per_xcd, int nchunk) {
  using T = C<R>;
  using V4 = typename R4<R>::type;
  constexpr int RT = RC / NS;                   // right-hand sides per lane
  constexpr int U = RC * (int)sizeof(T) / 16;   // 16-byte units per node and chunk
  constexpr int UP = U + 1;                     // units per node in LDS: odd, conflict-free
  constexpr int HX = TX + 2, HY = TY + 2;
  constexpr int NU = HX * HY * U;
  constexpr int NXR = (NU + NTHREADS - 1) / NTHREADS;
  constexpr int CPU = 16 / (int)sizeof(T);      // complex values per 16-byte unit
  static_assert(RT % CPU == 0 || CPU % RT == 0, "lane share of a chunk");
  static_assert(HX * HY <= NTHREADS, "one field node per thread");
  __shared__ __align__(16) float4 xs[HY][HX][UP];
  __shared__ R fw[3][3][HY][HX];   // ring slot, shell (face, edge, corner) mass weight
  __shared__ T fm[3][HY][HX];      // ring slot, m~
  // PML tiles: x factors per lx, y factors per ly, z factors of the planes
  // k0 - 2 .. k0 + TZ + 1; ring slot, S at the node
  __shared__ T fxs[PML ? TX : 1][9], fys[PML ? TY : 1][9], fzs[PML ? TZ + 4 : 1][9];
  __shared__ T fS[PML ? 3 : 1][PML ? HY : 1][PML ? HX : 1];

  const int bid = blockIdx.x;
  const int item = (bid % NXCD) * per_xcd + bid / NXCD;
  if (item >= nitems) return;
  // tile: columns [i0, i0 + TX) x [j0, j0 + TY), planes [k0, kend), kend - k0 <= TZ
  const int4 tl = tiles[item / nchunk];
  const int chunk = item % nchunk;
  const int i0 = tl.x, j0 = tl.y, k0 = tl.z, kend = tl.w;
  const int c0 = c_first + chunk * RC;
  const int tid = threadIdx.x;
  const int part = tid % NS, nl = tid / NS;
  const int lx = nl % TX, ly = nl / TX;
  const int gi = i0 + lx, gj = j0 + ly;
  const bool inside = gi < nx && gj < ny;
  // the output plane (p - 1 + ol) whose couplings this lane forms
  const int ol = part < 3 ? part : 1;
  const R om2 = (R)op.om2;
  const R W1 = (R)op.W1, W2 = (R)op.W2, W3 = (R)op.W3;

  if constexpr (PML) {
    for (int q = tid; q < (TX + TY + TZ + 4) * 9; q += NTHREADS) {
      const int l = q / 9, f = q % 9;
      if (l < TX) fxs[l][f] = op.fx[min(i0 + l, nx - 1) * 9 + f];
      else if (l < TX + TY) fys[l - TX][f] = op.fy[min(j0 + l - TX, ny - 1) * 9 + f];
      else fzs[l - TX - TY][f] = op.fz[min(max(k0 - 2 + l - TX - TY, 0), nz - 1) * 9 + f];
    }
  }

  // next plane of x and of node fields, staged in registers
  float4 xr[NXR];
  V4 f4r;
  R fir;
  T fsr;
  auto fetch_x = [&](int kk) {
    const bool kin = kk >= 0 && kk < nz;
#pragma unroll
    for (int j = 0; j < NXR; ++j) {
      const int q = tid + j * NTHREADS;
      const int u = q % U, hn = q / U;
      const int hi = i0 + hn % HX - 1, hj = j0 + hn / HX - 1;
      xr[j] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (q < NU && kin && hi >= 0 && hi < nx && hj >= 0 && hj < ny)
        xr[j] = reinterpret_cast<const float4*>(x + (((long long)kk * ny + hj) * nx + hi) * s + c0)[u];
    }
  };
  auto fetch_f = [&](int kk) {
    const int hi = i0 + tid % HX - 1, hj = j0 + tid / HX - 1;
    f4r.x = 0; f4r.y = 0; f4r.z = 0; f4r.w = 0;
    fir = 0;
    if constexpr (PML) fsr = mk<R>(1, 0);
    if (tid < HX * HY && kk >= 0 && kk < nz && hi >= 0 && hi < nx && hj >= 0 && hj < ny) {
      const long long g = ((long long)kk * ny + hj) * nx + hi;
      f4r = op.f4[g];
      fir = op.fim[g];
      if constexpr (PML)
        fsr = cmul(cmul(op.fx[hi * 9 + FN(0)], op.fy[hj * 9 + FN(0)]), op.fz[kk * 9 + FN(0)]);
    }
  };
  auto stash_x = [&]() {
#pragma unroll
    for (int j = 0; j < NXR; ++j) {
      const int q = tid + j * NTHREADS;
      if (q < NU) {
        const int u = q % U, hn = q / U;
        xs[hn / HX][hn % HX][u] = xr[j];
      }
    }
  };
  auto stash_f = [&](int slot) {
    if (tid < HX * HY) {
      const int hx = tid % HX, hy = tid / HX;
      fw[slot][0][hy][hx] = f4r.x;
      fw[slot][1][hy][hx] = f4r.y;
      fw[slot][2][hy][hx] = f4r.z;
      fm[slot][hy][hx] = mk<R>(f4r.w, fir);
      if constexpr (PML) fS[slot][hy][hx] = fsr;
    }
  };

  // outputs of planes p - 1, p, p + 1 of this lane's node and right-hand sides
  T acc[3][RT];
#pragma unroll
  for (int o = 0; o < 3; ++o)
#pragma unroll
    for (int q = 0; q < RT; ++q) acc[o][q] = cz<R>();

  // apply plane p to the outputs it couples to (o = 0, 1, 2: planes p - 1,
  // p, p + 1; the first and last steps of the march feed one of them)
  auto step = [&](int p, auto mode_tag) {
    constexpr int MODE = decltype(mode_tag)::value;
    constexpr int OLO = MODE == FIRST ? 2 : 0, OHI = MODE == LAST ? 0 : 2;
    const int cx = lx + 1, cy = ly + 1;
    const int sp = (p + 3) % 3;
    // this lane's output plane: own fields, offset of plane p seen from it
    const int so = (p + 2 + ol) % 3;
    const int ez = 1 - ol;
    const bool mid = ez == 0;
    const T mo = fm[so][cy][cx];
    const R wm0 = (R)1 - (R)6 * fw[so][0][cy][cx] - (R)12 * fw[so][1][cy][cx] -
                  (R)8 * fw[so][2][cy][cx];
    T So, zR, zH, zN0;
    if constexpr (PML) {
      So = fS[so][cy][cx];
      const T* fz = fzs[p - k0 + ol + 1];   // plane p - 1 + ol
      zR = fz[FR(ez)];
      zH = fz[FH(ez)];
      zN0 = fz[FN(0)];
    }
    const R sz = mid ? (R)-1 : (R)1;
    // stiffness of a PML-free tile per shell: centre, face, edge, corner
    const R st[4] = {-(6 * W1 + 24 * W2 + 24 * W3), W1 - 4 * W3, 2 * W2 + 2 * W3, 3 * W3};
    static_for<9>([&](auto E) {
      constexpr int ex = decltype(E)::value % 3 - 1, ey = decltype(E)::value / 3 - 1;
      constexpr int t0 = (ex != 0) + (ey != 0);
      // this lane's coupling: shell t = t0 (own plane) or t0 + 1
      const int t = t0 + (mid ? 0 : 1);
      const T mn = fm[sp][cy + ey][cx + ex];
      T c;
      if (t == 0) {
        // the centre: only the middle lane of the centre column
        c = csc<R>(mo, om2 * wm0);
        if constexpr (PML) c = cmul(c, So);
      } else {
        const int sh = t > 0 ? t - 1 : 0;   // (t = 0 takes the other branch)
        const R wsum = fw[so][sh][cy][cx] + fw[sp][sh][cy + ey][cx + ex];
        if constexpr (PML) {
          const T Sn = fS[sp][cy + ey][cx + ex];
          c = csc<R>(cmul(cadd(mo, mn), cadd(So, Sn)), om2 / (R)8 * wsum);
        } else {
          c = csc<R>(cadd(mo, mn), om2 / (R)4 * wsum);
        }
      }
      if constexpr (PML) {
        const T* fX = fxs[lx];
        const T* fY = fys[ly];
        const T Rx = fX[FR(ex)], Hx = fX[FH(ex)], Ry = fY[FR(ey)], Hy = fY[FH(ey)];
        constexpr R sx = ex ? 1 : -1, sy = ey ? 1 : -1;
        const T Qxy = cadd(csc<R>(cmul(Rx, Hy), sx), csc<R>(cmul(Ry, Hx), sy));
        // cube-centre family
        T v = csc<R>(cadd(cmul(zH, Qxy), csc<R>(cmul(zR, cmul(Hx, Hy)), sz)), W3);
        // in-plane families: (x, y) only for the own plane
        const T zN0m = mid ? zN0 : cz<R>();
        T ip = cmul(zN0m, Qxy);
        if constexpr (ey == 0)
          ip = cadd(ip, cmul(fY[FN(0)], cadd(csc<R>(cmul(Rx, zH), sx), csc<R>(cmul(zR, Hx), sz))));
        if constexpr (ex == 0)
          ip = cadd(ip, cmul(fX[FN(0)], cadd(csc<R>(cmul(Ry, zH), sy), csc<R>(cmul(zR, Hy), sz))));
        v = cadd(v, csc<R>(ip, W2));
        // axis families: x and y only for the own plane
        T ax = cz<R>();
        if constexpr (ey == 0) ax = cadd(ax, csc<R>(cmul(Rx, cmul(fY[FN(0)], zN0m)), sx));
        if constexpr (ex == 0) ax = cadd(ax, csc<R>(cmul(Ry, cmul(fX[FN(0)], zN0m)), sy));
        if constexpr (ex == 0 && ey == 0)
          ax = cadd(ax, csc<R>(cmul(zR, cmul(fX[FN(0)], fY[FN(0)])), sz));
        c = cadd(c, cadd(v, csc<R>(ax, W1)));
      } else {
        // (selected with compile-time indices: a runtime index would put st
        // in LDS)
        c.x += mid ? st[t0] : st[t0 + 1];
      }
      // the quad's couplings of the three output planes
      T cc[3];
      if constexpr (OLO <= 0 && 0 <= OHI) cc[0] = quad_bcast_c<0>(c);
      if constexpr (OLO <= 1 && 1 <= OHI) cc[1] = quad_bcast_c<1>(c);
      if constexpr (OLO <= 2 && 2 <= OHI) cc[2] = quad_bcast_c<2>(c);
#pragma unroll
      for (int q = 0; q < RT; ++q) {
        const T xv = reinterpret_cast<const T*>(
            &xs[cy + ey][cx + ex][part * (RT / CPU) + q / CPU])[q % CPU];
#pragma unroll
        for (int o = OLO; o <= OHI; ++o) cfma(acc[o][q], cc[o], xv);
      }
      // one neighbour column at a time: left free, the compiler hoists every
      // LDS read of the plane, and sinks the products into the completed
      // output into its conditional store, keeping all of them live
#pragma unroll
      for (int o = OLO; o <= OHI; ++o)
#pragma unroll
        for (int q = 0; q < RT; ++q) pin(acc[o][q]);
      __builtin_amdgcn_sched_barrier(0);
    });
  };

  // output plane k is complete once plane k + 1 has been applied
  auto flush = [&](int k) {
    if (inside && k >= k0 && k < kend) {
      const long long o = (((long long)k * ny + gj) * nx + gi) * s + c0 + part * RT;
#pragma unroll
      for (int q = 0; q < RT; ++q) {
        double2 out = make_double2((double)acc[0][q].x, (double)acc[0][q].y);
        if (b) out = csub(b[o + q], out);
        if constexpr (std::is_same<Y, double2>::value) {
          y[o + q] = out;
        } else {
          // single-precision output (no b): the value is already an FP32 one
          y[o + q] = make_float2((float)out.x, (float)out.y);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < RT; ++q) {
      acc[0][q] = acc[1][q];
      acc[1][q] = acc[2][q];
      acc[2][q] = cz<R>();
    }
  };

  // plane p: its x values and the fields of plane p + 1 enter LDS, the next
  // plane's loads are issued, then plane p is applied.  A quad works on one
  // node and the DPP exchange reads its lanes, so every quad steps (the
  // results of nodes outside the grid are dropped by flush).
  auto advance = [&](int p) {
    stash_x();
    stash_f((p + 4) % 3);
    __syncthreads();
    if (p < kend) fetch_x(p + 1);
    fetch_f(p + 2);
  };
  fetch_f(k0 - 1);
  stash_f((k0 + 2) % 3);
  fetch_f(k0);
  fetch_x(k0 - 1);
  advance(k0 - 1);
  step(k0 - 1, std::integral_constant<int, FIRST>());
  flush(k0 - 2);
  __syncthreads();
  for (int p = k0; p < kend; ++p) {
    advance(p);
    step(p, std::integral_constant<int, MID>());
    flush(p - 1);
    __syncthreads();
  }
  advance(kend);
  step(kend, std::integral_constant<int, LAST>());
  flush(kend - 1);
}

template <typename R>
__global__ void mass_fields_kernel(const double* w7, const double2* mt, long long n,
                                   typename R4<R>::type* f4, R* fim) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  typename R4<R>::type f;
  f.x = (R)w7[i * 7 + 4];
  f.y = (R)w7[i * 7 + 5];
  f.z = (R)w7[i * 7 + 6];
  f.w = (R)mt[i].x;
  f4[i] = f;
  fim[i] = (R)mt[i].y;
}

template <typename R, bool PML, int RC, typename Y>
void launch_chunks(const StencilMF<R>& op, const C<R>* x, const double2* b, Y* y, int nx,
                   int ny, int nz, int s, int c_first, int nchunk, hipStream_t st) {
  const int lo = PML ? op.nplain : 0, hi = PML ? op.ntiles : op.nplain;
  if (hi == lo || nchunk == 0) return;
  const int nitems = (hi - lo) * nchunk;
  const int per_xcd = (nitems + NXCD - 1) / NXCD;
  hipLaunchKernelGGL((stencil_mf_kernel<R, PML, RC, Y>), dim3((unsigned)(per_xcd * NXCD)),
                     dim3(NTHREADS), 0, st, op, op.tiles + lo, x, b, y, nx, ny, nz, s, c_first,
                     nitems, per_xcd, nchunk);
}

template <typename R, bool PML, typename Y>
void launch_kind(const StencilMF<R>& op, const C<R>* x, const double2* b, Y* y, int nx,
                 int ny, int nz, int s, hipStream_t st) {
  // chunks of the widest width, then narrower chunks for the rest (s is a
  // multiple of 8)
  constexpr int RC = MfChunk<R, PML>::RC;
  const int full = s / RC;
  int c = full * RC;
  launch_chunks<R, PML, RC, Y>(op, x, b, y, nx, ny, nz, s, 0, full, st);
  if constexpr (RC > 16) {
    if (s - c >= 16) {
      launch_chunks<R, PML, 16, Y>(op, x, b, y, nx, ny, nz, s, c, 1, st);
      c += 16;
    }
  }
  if constexpr (RC > 8) {
    if (s - c >= 8) launch_chunks<R, PML, 8, Y>(op, x, b, y, nx, ny, nz, s, c, 1, st);
  }
}

}  // namespace

template <typename R>
void launch_mass_fields(const double* w7, const double2* mt, long long n,
                        typename R4<R>::type* f4, R* fim, hipStream_t st) {
  const int bs = 256;
  hipLaunchKernelGGL((mass_fields_kernel<R>), dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, st,
                     w7, mt, n, f4, fim);
}

void stencil_mf_tiles(const int lo[3], const int hi[3], int nx, int ny, int nz,
                      std::vector<int>& tiles, int& nplain) {
  const int n[3] = {nx, ny, nz}, t[3] = {TX, TY, TZ};
  std::vector<int> pml;
  tiles.clear();
  for (int k0 = 0; k0 < nz; k0 += TZ)
    for (int j0 = 0; j0 < ny; j0 += TY)
      for (int i0 = 0; i0 < nx; i0 += TX) {
        const int b0[3] = {i0, j0, k0};
        bool plain = true;
        for (int a = 0; a < 3; ++a)
          plain = plain && b0[a] >= lo[a] && std::min(b0[a] + t[a], n[a]) <= hi[a];
        std::vector<int>& v = plain ? tiles : pml;
        v.insert(v.end(), {i0, j0, k0, std::min(k0 + TZ, nz)});
      }
  nplain = (int)(tiles.size() / 4);
  tiles.insert(tiles.end(), pml.begin(), pml.end());
}

template <typename R, typename Y>
void launch_stencil_mf(const StencilMF<R>& op, const C<R>* x, const double2* b, Y* y, int nx,
                       int ny, int nz, int s, hipStream_t st) {
  static_assert(RHS_ALIGN == 8, "chunk widths cover multiples of 8");
  launch_kind<R, false, Y>(op, x, b, y, nx, ny, nz, s, st);
  launch_kind<R, true, Y>(op, x, b, y, nx, ny, nz, s, st);
}

template void launch_mass_fields<float>(const double*, const double2*, long long, float4*, float*,
                                        hipStream_t);
template void launch_mass_fields<double>(const double*, const double2*, long long, double4*,
                                         double*, hipStream_t);
template void launch_stencil_mf<float, double2>(const StencilMF<float>&, const float2*,
                                                const double2*, double2*, int, int, int, int,
                                                hipStream_t);
template void launch_stencil_mf<float, float2>(const StencilMF<float>&, const float2*,
                                               const double2*, float2*, int, int, int, int,
                                               hipStream_t);
template void launch_stencil_mf<double, double2>(const StencilMF<double>&, const double2*,
                                                 const double2*, double2*, int, int, int, int,
                                                 hipStream_t);

}  // namespace oras
