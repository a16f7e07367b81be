// Multi-RHS 27-point stencil apply y = A x (or the residual y = b - A x).
//
// Paper sec. 2.2: the Krylov iteration applies A to a block of right-hand
// sides; sec. 2.3: A is the compact 27-point stencil (one row per grid node,
// couplings to the 3x3x3 neighbourhood).  Vectors use the right-hand-side
// fastest layout [node][s] so every neighbour access reads s contiguous
// complex values; the 27 coefficients of a node are stored structure of
// arrays, slot e = (ez+1)*9 + (ey+1)*3 + (ex+1), so consecutive nodes read
// consecutive addresses.
//
// A work-group owns a TX x TY tile of one z-plane and a chunk of RC
// right-hand sides, and marches the tile through TZ planes.  The x values of
// the tile and its one-node halo are staged in LDS as a three-plane ring (16
// byte vector loads), so each x value is read from memory about once per
// plane sweep.  Two threads share a node (RC / 2 right-hand sides each), so a
// coefficient load serves RC / 2 products per thread and the two loads of a
// node coalesce into one request.  The chunks of one tile are
// given work-group ids that the hardware places on the same XCD, so they
// share the tile's coefficients (and halo) through that XCD's L2.
#include "oras_internal.h"

namespace oras {

namespace {

constexpr int TX = 16;
constexpr int TY = 16;
constexpr int TZ = 8;
constexpr int NXCD = 8;

template <typename R> struct StencilChunk;
// Per precision (chosen by measurement on gfx950 at 160^3 x 32 right-hand
// sides): chunk width, whether the in-plane neighbour rows are unrolled, and
// whether the next x plane is fetched into registers ahead of the arithmetic.
template <> struct StencilChunk<float> {
  static constexpr int RC = 8;
  static constexpr bool EY = true, PIPE = false;
};
template <> struct StencilChunk<double> {
  static constexpr int RC = 4;
  static constexpr bool EY = false, PIPE = true;
};
constexpr int NSPLIT = 2;                 // threads per node
constexpr int NTHREADS = TX * TY * NSPLIT;

template <typename R>
__global__ void __launch_bounds__(NTHREADS)
stencil_kernel(const C<R>* __restrict__ coef, const C<R>* __restrict__ x,
               const double2* __restrict__ b, double2* __restrict__ y, int nx, int ny, int nz,
               int s, int ntx, int nty, int ntiles, int nchunk) {
  using T = C<R>;
  constexpr int RC = StencilChunk<R>::RC;
  constexpr bool UNROLL_EY = StencilChunk<R>::EY;
  constexpr int U = RC * (int)sizeof(T) / 16;   // 16-byte units per node and chunk
  constexpr int HX = TX + 2, HY = TY + 2;
  // x plane ring, 16-byte unit u of a node's chunk slowest within a row, rows
  // padded to HXP units: a thread's two units sit in rows of units that are
  // 2 HXP apart, which keeps each 16-byte LDS read free of bank conflicts
  constexpr int HXP = HX + 2;
  __shared__ __align__(16) float4 ring[3][HY][U][HXP];

  // work-group id -> (tile, chunk): the chunks of a tile on one XCD, adjacent in time
  const int bid = blockIdx.x, r = bid / NXCD;
  const int tile = (r / nchunk) * NXCD + bid % NXCD;
  const int chunk = r % nchunk;
  if (tile >= ntiles) return;
  const int bx = tile % ntx, by = (tile / ntx) % nty, bz = tile / (ntx * nty);
  const int i0 = bx * TX, j0 = by * TY, k0 = bz * TZ;
  const int c0 = chunk * RC;
  const long long n = (long long)nx * ny * nz;
  constexpr int RT = RC / NSPLIT;            // right-hand sides per thread
  const int tid = threadIdx.x;
  const int part = tid % NSPLIT, nl = tid / NSPLIT;
  const int lx = nl % TX, ly = nl / TX;

  const int gi = i0 + lx, gj = j0 + ly;
  const bool inside = gi < nx && gj < ny;
  // one output node (all of this thread's right-hand sides) of plane k
  auto compute = [&](int k) {
    const long long node = ((long long)k * ny + gj) * nx + gi;
    T acc[RT];
#pragma unroll
    for (int c = 0; c < RT; ++c) {
      acc[c].x = 0;
      acc[c].y = 0;
    }
    auto row = [&](int slot, int ez, int ey) {
#pragma unroll
      for (int ex = -1; ex <= 1; ++ex) {
        const T a = coef[eidx(ex, ey, ez) * n + node];
        T xv[RT];
        constexpr int CPU = 16 / (int)sizeof(T);   // complex values per 16-byte unit
#pragma unroll
        for (int c = 0; c < RT; ++c)
          xv[c] = reinterpret_cast<const T*>(
              &ring[slot][ly + 1 + ey][part * (RT / CPU) + c / CPU][lx + 1 + ex])[c % CPU];
#pragma unroll
        for (int c = 0; c < RT; ++c) cfma(acc[c], a, xv[c]);
      }
    };
    // the neighbour loops are unrolled only partly: unrolling all 27 makes
    // the compiler hoist every load and exhausts the register file
#pragma unroll 1
    for (int ez = -1; ez <= 1; ++ez) {
      const int slot = (k + ez + 3) % 3;
      if constexpr (UNROLL_EY) {
#pragma unroll
        for (int ey = -1; ey <= 1; ++ey) row(slot, ez, ey);
      } else {
#pragma unroll 1
        for (int ey = -1; ey <= 1; ++ey) row(slot, ez, ey);
      }
    }
    const long long o = node * s + c0 + part * RT;
#pragma unroll
    for (int c = 0; c < RT; ++c) {
      double2 out = make_double2((double)acc[c].x, (double)acc[c].y);
      if (b) out = csub(b[o + c], out);
      y[o + c] = out;
    }
  };

  // a plane of x values (tile + halo, this chunk) in 16-byte units
  constexpr int NU = HX * HY * U;
  const int kend = min(k0 + TZ, nz);
  if constexpr (!StencilChunk<R>::PIPE) {
    // plane k + 1 staged right before plane k is computed
    auto load_plane = [&](int kk, int slot) {
      for (int q = tid; q < NU; q += NTHREADS) {
        const int u = q % U, hn = q / U;
        const int hx = hn % HX, hy = hn / HX;
        const int hi = i0 + hx - 1, hj = j0 + hy - 1;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (kk >= 0 && kk < nz && hi >= 0 && hi < nx && hj >= 0 && hj < ny)
          v = reinterpret_cast<const float4*>(x + (((long long)kk * ny + hj) * nx + hi) * s + c0)[u];
        ring[slot][hy][u][hx] = v;
      }
    };
    load_plane(k0 - 1, (k0 + 2) % 3);
    load_plane(k0, k0 % 3);
    for (int k = k0; k < kend; ++k) {
      load_plane(k + 1, (k + 1) % 3);
      __syncthreads();
      if (inside) compute(k);
      __syncthreads();
    }
  } else {
    // planes k0 - 1 .. k0 + 1 staged up front; plane k + 2 is fetched into
    // registers before plane k is computed and stored after it, so its
    // memory latency overlaps the arithmetic
    constexpr int PER = (NU + NTHREADS - 1) / NTHREADS;
    float4 pre[PER];
    auto fetch = [&](int kk) {
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int q = tid + i * NTHREADS;
        pre[i] = make_float4(0.f, 0.f, 0.f, 0.f);
        const int u = q % U, hn = q / U;
        const int hi = i0 + hn % HX - 1, hj = j0 + hn / HX - 1;
        if (q < NU && kk >= 0 && kk < nz && hi >= 0 && hi < nx && hj >= 0 && hj < ny)
          pre[i] = reinterpret_cast<const float4*>(x + (((long long)kk * ny + hj) * nx + hi) * s + c0)[u];
      }
    };
    auto stash = [&](int slot) {
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int q = tid + i * NTHREADS;
        const int u = q % U, hn = q / U;
        if (q < NU) ring[slot][hn / HX][u][hn % HX] = pre[i];
      }
    };
    fetch(k0 - 1);
    stash((k0 + 2) % 3);
    fetch(k0);
    stash(k0 % 3);
    fetch(k0 + 1);
    stash((k0 + 1) % 3);
    for (int k = k0; k < kend; ++k) {
      const bool more = k + 1 < kend;
      if (more) fetch(k + 2);
      __syncthreads();
      if (inside) compute(k);
      __syncthreads();
      if (more) stash((k + 2) % 3);
    }
  }
}

}  // namespace

// s must be a multiple of RHS_ALIGN (every internal vector is padded so).
template <typename R>
void launch_stencil(const C<R>* coef, const C<R>* x, const double2* b, double2* y, int nx, int ny,
                    int nz, int s, hipStream_t st) {
  constexpr int RC = StencilChunk<R>::RC;
  static_assert(RHS_ALIGN % RC == 0, "chunk must divide the right-hand-side padding");
  const int ntx = (nx + TX - 1) / TX, nty = (ny + TY - 1) / TY, ntz = (nz + TZ - 1) / TZ;
  const int ntiles = ntx * nty * ntz;
  const int nchunk = s / RC;
  if (nchunk == 0) return;
  const long long nblk = (long long)(ntiles + NXCD - 1) / NXCD * NXCD * nchunk;
  hipLaunchKernelGGL((stencil_kernel<R>), dim3((unsigned)nblk), dim3(NTHREADS), 0, st, coef, x, b,
                     y, nx, ny, nz, s, ntx, nty, ntiles, nchunk);
}

template void launch_stencil<float>(const float2*, const float2*, const double2*, double2*, int,
                                    int, int, int, hipStream_t);
template void launch_stencil<double>(const double2*, const double2*, const double2*, double2*,
                                     int, int, int, int, hipStream_t);

}  // namespace oras
