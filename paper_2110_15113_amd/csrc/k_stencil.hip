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
// A work-group owns a TX x TY tile of one z-plane for RC right-hand sides and
// marches it through TZ planes; the x values of the tile and its one-node
// halo are staged in LDS as a three-plane ring, so each x value is read from
// HBM about once per plane sweep instead of 27 times.
#include "oras_internal.h"

namespace oras {

namespace {

constexpr int TX = 16;
constexpr int TY = 8;
constexpr int TZ = 8;

template <typename R, int RC>
__global__ void __launch_bounds__(TX * TY * RC)
stencil_kernel(const C<R>* __restrict__ coef, const C<R>* __restrict__ x,
               const double2* __restrict__ b, double2* __restrict__ y, int nx, int ny, int nz,
               int s) {
  using T = C<R>;
  __shared__ T ring[3][TY + 2][TX + 2][RC];
  const long long n = (long long)nx * ny * nz;
  const int tid = threadIdx.x;
  const int c = tid % RC;
  const int lx = (tid / RC) % TX;
  const int ly = tid / (RC * TX);
  // right-hand-side chunks of one tile are adjacent block indices, so they run
  // together and share the tile's coefficients through L2
  const int nchunk = (s + RC - 1) / RC;
  const int chunk = blockIdx.x % nchunk;
  const int tile = blockIdx.x / nchunk;
  const int ntx = (nx + TX - 1) / TX;
  const int bx = tile % ntx;
  const int by = tile / ntx;
  const int i0 = bx * TX, j0 = by * TY;
  const int k0 = blockIdx.y * TZ;
  const int c0 = chunk * RC;
  const int cc = c0 + c;
  const int halo = (TX + 2) * (TY + 2);
  const int nthreads = TX * TY * RC;

  auto load_plane = [&](int kk, int slot) {
    for (int q = tid; q < halo * RC; q += nthreads) {
      const int r = q % RC;
      const int hx = (q / RC) % (TX + 2);
      const int hy = (q / RC) / (TX + 2);
      const int gi = i0 + hx - 1, gj = j0 + hy - 1;
      T v;
      v.x = 0;
      v.y = 0;
      if (kk >= 0 && kk < nz && gi >= 0 && gi < nx && gj >= 0 && gj < ny && c0 + r < s)
        v = x[(((long long)kk * ny + gj) * nx + gi) * s + c0 + r];
      ring[slot][hy][hx][r] = v;
    }
  };

  load_plane(k0 - 1, (k0 + 2) % 3);
  load_plane(k0, k0 % 3);
  const int kend = min(k0 + TZ, nz);
  for (int k = k0; k < kend; ++k) {
    load_plane(k + 1, (k + 1) % 3);
    __syncthreads();
    const int gi = i0 + lx, gj = j0 + ly;
    if (gi < nx && gj < ny && cc < s) {
      const long long node = ((long long)k * ny + gj) * nx + gi;
      T acc;
      acc.x = 0;
      acc.y = 0;
#pragma unroll
      for (int ez = -1; ez <= 1; ++ez) {
        const int slot = (k + ez + 3) % 3;
#pragma unroll
        for (int ey = -1; ey <= 1; ++ey)
#pragma unroll
          for (int ex = -1; ex <= 1; ++ex) {
            const T a = coef[eidx(ex, ey, ez) * n + node];
            const T v = ring[slot][ly + 1 + ey][lx + 1 + ex][c];
            cfma(acc, a, v);
          }
      }
      double2 out = make_double2((double)acc.x, (double)acc.y);
      const long long o = node * s + cc;
      if (b) out = csub(b[o], out);
      y[o] = out;
    }
    __syncthreads();
  }
}

}  // namespace

template <typename R>
void launch_stencil(const C<R>* coef, const C<R>* x, const double2* b, double2* y, int nx, int ny,
                    int nz, int s, hipStream_t st) {
  const int ntx = (nx + TX - 1) / TX, nty = (ny + TY - 1) / TY;
  const int ntz = (nz + TZ - 1) / TZ;
  if (s % 4 == 0 || s > 4) {
    constexpr int RC = 4;
    dim3 grid(ntx * nty * ((s + RC - 1) / RC), ntz);
    hipLaunchKernelGGL((stencil_kernel<R, RC>), grid, dim3(TX * TY * RC), 0, st, coef, x, b, y,
                       nx, ny, nz, s);
  } else {
    constexpr int RC = 1;
    dim3 grid(ntx * nty * s, ntz);
    hipLaunchKernelGGL((stencil_kernel<R, RC>), grid, dim3(TX * TY * RC), 0, st, coef, x, b, y,
                       nx, ny, nz, s);
  }
}

template void launch_stencil<float>(const float2*, const float2*, const double2*, double2*, int,
                                    int, int, int, hipStream_t);
template void launch_stencil<double>(const double2*, const double2*, const double2*, double2*,
                                     int, int, int, int, hipStream_t);

}  // namespace oras
