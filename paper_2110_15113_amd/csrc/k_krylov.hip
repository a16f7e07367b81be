// FP64 kernels of pseudo-block flexible GMRES (paper sec. 2.1: right
// preconditioning; sec. 2.2: flexible variant and pseudo-block processing;
// sec. 3.2: classical Gram-Schmidt), plus layout conversion, point sources,
// receiver sampling and the adjoint gradient.
//
// Internal vectors are [node][s] complex128 (right-hand sides fastest).  The
// Arnoldi basis is stored unnormalised: v_i = scale_i * V_i with a per-column
// real factor, so normalising a new basis vector costs no extra pass.
// All reductions are two-stage with a fixed order (per-block partial sums,
// then a serial sum over blocks), so results are bitwise reproducible.
#include "oras_internal.h"

namespace oras {

namespace {

__global__ void to_internal_kernel(const double2* __restrict__ src, double2* __restrict__ dst,
                                   long long n, int nrhs, int s, int conj) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * s) return;
  const long long node = idx / s;
  const int c = (int)(idx % s);
  double2 v = make_double2(0.0, 0.0);
  if (c < nrhs) {
    v = src[(long long)c * n + node];
    if (conj) v.y = -v.y;
  }
  dst[idx] = v;
}

// [n][s] -> [nrhs][n] through an LDS tile of 64 nodes x 32 columns, so that
// both the reads (a node's columns) and the writes (a column's nodes) are
// contiguous runs.
constexpr int TR_NODES = 64, TR_COLS = 32;
__global__ void __launch_bounds__(256)
from_internal_kernel(const double2* __restrict__ src, double2* __restrict__ dst, long long n,
                     int nrhs, int s, int conj) {
  __shared__ double2 tile[TR_NODES][TR_COLS + 1];
  const long long node0 = (long long)blockIdx.x * TR_NODES;
  const int c0 = blockIdx.y * TR_COLS;
  for (int i = threadIdx.x; i < TR_NODES * TR_COLS; i += 256) {
    const int r = i / TR_COLS, j = i % TR_COLS;
    const long long node = node0 + r;
    const int c = c0 + j;
    if (node < n && c < nrhs) tile[r][j] = src[node * s + c];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < TR_NODES * TR_COLS; i += 256) {
    const int j = i / TR_NODES, r = i % TR_NODES;
    const long long node = node0 + r;
    const int c = c0 + j;
    if (node < n && c < nrhs) {
      double2 v = tile[r][j];
      if (conj) v.y = -v.y;
      dst[(long long)c * n + node] = v;
    }
  }
}

// Sum over the lanes of a 64-lane wave that share lane % s (s a power of
// two): a butterfly over the lane offsets >= s, fixed order, no barrier.
// Lane l < s of the wave holds the sum (every lane does, in some order).
__device__ inline double wave_sum_stride(double v, int s) {
  for (int o = 32; o >= s; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// The threads of a work-group that share a column (thread t holds column
// t % s) meet in one wave at power-of-two lane distances when s is a power of
// two below 64 (the work-group is then 256 threads).
__device__ inline bool wave_columns(int s) { return s < 64 && (s & (s - 1)) == 0; }

// Column sums of a work-group whose thread t holds column t % s, G groups of
// s threads: wave butterflies and the waves' sums in wave order through LDS
// when the columns meet in waves, else the G group sums in order.
__device__ inline void block_reduce_store(double* lds, double v, int s, int G, double* out) {
  const int tid = threadIdx.x;
  if (wave_columns(s)) {
    v = wave_sum_stride(v, s);
    if ((tid & 63) < s) lds[(tid >> 6) * s + (tid & 63)] = v;
  } else {
    lds[tid] = v;
  }
  __syncthreads();
  if (tid < s) {
    double acc = 0.0;
    if (wave_columns(s)) {
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) acc += lds[w * s + tid];
    } else {
      for (int g = 0; g < G; ++g) acc += lds[g * s + tid];
    }
    *out = acc;
  }
  __syncthreads();
}


// The basis vectors and the updated w are streamed (each pass touches
// gigabytes before anything is read again): non-temporal loads and stores
// keep them out of the caches' way (Gram-Schmidt 0.666 -> 0.636 s per
// config-5 solve).
typedef double f64x2nt __attribute__((ext_vector_type(2)));
__device__ inline double2 ldnt2(const double2* p) {
  const f64x2nt v = __builtin_nontemporal_load(reinterpret_cast<const f64x2nt*>(p));
  return make_double2(v.x, v.y);
}
__device__ inline void stnt2(double2* p, double2 v) {
  f64x2nt u; u.x = v.x; u.y = v.y;
  __builtin_nontemporal_store(u, reinterpret_cast<f64x2nt*>(p));
}

__global__ void colnorm2_kernel(const double2* __restrict__ x, long long n, int s,
                                double* __restrict__ partial) {
  __shared__ double lds[256];
  const int G = blockDim.x / s;
  const int c = threadIdx.x % s, g = threadIdx.x / s;
  double acc = 0.0;
  for (long long node = (long long)blockIdx.x * G + g; node < n; node += (long long)gridDim.x * G) {
    const double2 v = x[node * s + c];
    acc += v.x * v.x + v.y * v.y;
  }
  block_reduce_store(lds, acc, s, G, partial + (long long)blockIdx.x * s + c);
}

// Fixed-order sum of 256 per-thread values (deterministic): a butterfly
// within each 64-lane wave, then the four wave sums in order through LDS.
__device__ inline double tree_sum(double* lds, double v) {
  v = wave_sum_stride(v, 1);
  __syncthreads();   // earlier readers of lds are done
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
  __syncthreads();
  return (lds[0] + lds[1]) + (lds[2] + lds[3]);
}

// out[c] = sqrt(sum over blocks of partial[blk][c]); one work-group per column
__global__ void __launch_bounds__(256) finish_norm_kernel(const double* __restrict__ partial,
                                                          int nblk, int s,
                                                          double* __restrict__ out) {
  __shared__ double lds[256];
  const int c = blockIdx.x;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 256) acc += partial[(long long)b * s + c];
  const double t = tree_sum(lds, acc);
  if (threadIdx.x == 0) out[c] = sqrt(t);
}

__device__ inline double2 as_c128(double2 v) { return v; }
__device__ inline double2 as_c128(float2 v) { return make_double2((double)v.x, (double)v.y); }

// partial[blk][i][c] = sum_nodes conj(V_i) w   for i < j1   (scale applied later).
// w is complex128, or complex64 when it comes from the single-precision
// stencil (whose values are FP32 ones: widening them is exact).
template <typename W>
__global__ void cgs_dot_kernel(const double2* __restrict__ V, long long vstride, int j1,
                               const W* __restrict__ w, long long n, int s,
                               double2* __restrict__ partial) {
  __shared__ double lre[8 * 256];
  __shared__ double lim[8 * 256];
  const int G = blockDim.x / s;
  const int c = threadIdx.x % s, g = threadIdx.x / s;
  for (int i0 = 0; i0 < j1; i0 += 8) {
    const int cnt = min(8, j1 - i0);
    double2 acc[8];
#pragma unroll
    for (int ii = 0; ii < 8; ++ii) acc[ii] = make_double2(0.0, 0.0);
    for (long long node = (long long)blockIdx.x * G + g; node < n;
         node += (long long)gridDim.x * G) {
      const double2 wv = as_c128(w[node * s + c]);
#pragma unroll
      for (int ii = 0; ii < 8; ++ii)
        if (ii < cnt) cfmaconj(acc[ii], ldnt2(&V[(long long)(i0 + ii) * vstride + node * s + c]), wv);
    }
    // column sums of the cnt basis vectors behind one barrier: butterflies
    // within each wave and the waves in order when the columns meet in
    // waves, else the G group sums in order
    const bool wc = wave_columns(s);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int ii = 0; ii < 8; ++ii) {
      if (ii < cnt) {
        if (wc) {
          const double re = wave_sum_stride(acc[ii].x, s), im = wave_sum_stride(acc[ii].y, s);
          if (lane < s) {
            lre[(ii * 4 + wave) * s + lane] = re;
            lim[(ii * 4 + wave) * s + lane] = im;
          }
        } else {
          lre[ii * 256 + threadIdx.x] = acc[ii].x;
          lim[ii * 256 + threadIdx.x] = acc[ii].y;
        }
      }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < cnt * s; q += blockDim.x) {
      const int ii = q / s, cc = q % s;
      double2 t = make_double2(0.0, 0.0);
      if (wc) {
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
          t.x += lre[(ii * 4 + w) * s + cc];
          t.y += lim[(ii * 4 + w) * s + cc];
        }
      } else {
        for (int g = 0; g < G; ++g) {
          t.x += lre[ii * 256 + g * s + cc];
          t.y += lim[ii * 256 + g * s + cc];
        }
      }
      partial[((long long)blockIdx.x * j1 + i0 + ii) * s + cc] = t;
    }
    __syncthreads();
  }
}

// h[i][c] = scale[i][c] * sum_blk partial   (i < j1); hs = h * scale (for the update)
// one work-group per (i, c), fixed-order tree over the block partials
__global__ void __launch_bounds__(256)
cgs_finish_dot_kernel(const double2* __restrict__ partial, int nblk, int j1, int s,
                      const double* __restrict__ scale, double2* __restrict__ h,
                      double2* __restrict__ hs) {
  __shared__ double lds[256];
  const int idx = blockIdx.x;
  const int i = idx / s, c = idx % s;
  double2 acc = make_double2(0.0, 0.0);
  for (int b = threadIdx.x; b < nblk; b += 256)
    acc = cadd(acc, partial[((long long)b * j1 + i) * s + c]);
  const double re = tree_sum(lds, acc.x);
  const double imv = tree_sum(lds, acc.y);
  if (threadIdx.x == 0) {
    const double sc = scale[idx];
    const double2 v = make_double2(re * sc, imv * sc);
    h[idx] = v;
    hs[idx] = cscale(v, sc);
  }
}

// wout = win - sum_i V_i hs_i (complex128; win complex128 in place, or the
// complex64 output of the single-precision stencil); partial[blk][c] = sum |wout|^2
template <typename W>
__global__ void cgs_update_kernel(const double2* __restrict__ V, long long vstride, int j1,
                                  const double2* __restrict__ hs, const W* win,
                                  double2* wout, long long n, int s,
                                  double* __restrict__ partial) {
  __shared__ double lds[256];
  const int G = blockDim.x / s;
  const int c = threadIdx.x % s, g = threadIdx.x / s;
  double acc = 0.0;
  for (long long node = (long long)blockIdx.x * G + g; node < n; node += (long long)gridDim.x * G) {
    double2 wv = as_c128(win[node * s + c]);
    for (int i = 0; i < j1; ++i) {
      const double2 v = ldnt2(&V[(long long)i * vstride + node * s + c]);
      const double2 hh = hs[i * s + c];
      cfms(wv, v, hh);
    }
    stnt2(&wout[node * s + c], wv);
    acc += wv.x * wv.x + wv.y * wv.y;
  }
  block_reduce_store(lds, acc, s, G, partial + (long long)blockIdx.x * s + c);
}

// One Arnoldi step per column: H column j, Givens rotation, residual estimate.
// H[(i * m + j) * s + c] for row i in 0..m, column j in 0..m-1.
__global__ void arnoldi_step_kernel(int j, int m, int s, const double* __restrict__ hnorm,
                                    const double2* __restrict__ h, double2* H, double* cs,
                                    double2* sn, double2* g, double* scale_next, int* jc,
                                    int* done, const double* __restrict__ bnorm, double tol,
                                    double* est) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= s) return;
  const double hn = hnorm[c];
  if (done[c]) {
    scale_next[c] = 0.0;
    return;
  }
  auto Hc = [&](int i, int jj) -> double2& { return H[((long long)i * m + jj) * s + c]; };
  for (int i = 0; i <= j; ++i) Hc(i, j) = h[i * s + c];
  Hc(j + 1, j) = make_double2(hn, 0.0);
  for (int i = 0; i < j; ++i) {
    const double ci = cs[i * s + c];
    const double2 si = sn[i * s + c];
    const double2 a = Hc(i, j), b = Hc(i + 1, j);
    double2 t = cadd(cscale(a, ci), cmul(si, b));
    double2 u = csub(cscale(b, ci), cmul(make_double2(si.x, -si.y), a));
    Hc(i, j) = t;
    Hc(i + 1, j) = u;
  }
  const double2 a = Hc(j, j), b = Hc(j + 1, j);
  const double na = hypot(a.x, a.y), nb = hypot(b.x, b.y);
  const double r = hypot(na, nb);
  double cj;
  double2 sj;
  if (na == 0.0) {
    cj = 0.0;
    sj = make_double2(1.0, 0.0);
  } else {
    cj = na / r;
    const double2 ua = make_double2(a.x / na, a.y / na);
    sj = cscale(cmul(ua, make_double2(b.x, -b.y)), 1.0 / r);
  }
  cs[j * s + c] = cj;
  sn[j * s + c] = sj;
  Hc(j, j) = cadd(cscale(a, cj), cmul(sj, b));
  Hc(j + 1, j) = make_double2(0.0, 0.0);
  const double2 gj = g[j * s + c];
  g[(j + 1) * s + c] = cmul(make_double2(-sj.x, sj.y), gj);
  g[j * s + c] = cscale(gj, cj);
  jc[c] = j + 1;
  const double2 gn = g[(j + 1) * s + c];
  const double e = hypot(gn.x, gn.y) / bnorm[c];
  est[c] = e;
  const bool fin = isfinite(hn) && isfinite(e);
  if (!fin) {
    done[c] = 2;           // numeric breakdown
    scale_next[c] = 0.0;
    return;
  }
  if (e <= tol || hn == 0.0) done[c] = 1;
  scale_next[c] = (hn > 0.0 && !done[c]) ? 1.0 / hn : 0.0;
}

__global__ void cycle_init_kernel(int s, int m, const double* __restrict__ beta,
                                  const int* __restrict__ conv, double2* g, double* scale0,
                                  int* jc, int* done) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= s) return;
  for (int i = 0; i <= m; ++i) g[i * s + c] = make_double2(0.0, 0.0);
  jc[c] = 0;
  if (conv[c]) {
    done[c] = 1;
    scale0[c] = 0.0;
  } else {
    done[c] = 0;
    g[c] = make_double2(beta[c], 0.0);
    scale0[c] = 1.0 / beta[c];
  }
}

__global__ void backsolve_kernel(int m, int s, const double2* __restrict__ H,
                                 const double2* __restrict__ g, const int* __restrict__ jc,
                                 double2* __restrict__ y) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= s) return;
  const int n = jc[c];
  for (int i = n - 1; i >= 0; --i) {
    double2 acc = g[i * s + c];
    for (int l = i + 1; l < n; ++l)
      acc = csub(acc, cmul(H[((long long)i * m + l) * s + c], y[l * s + c]));
    y[i * s + c] = cdiv(acc, H[((long long)i * m + i) * s + c]);
  }
}

template <typename Z>
__global__ void update_x_kernel(const Z* __restrict__ Zb, long long zstride, const double2* y,
                                const int* __restrict__ jc, double2* __restrict__ x, long long n,
                                int s) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * s) return;
  const int c = (int)(idx % s);
  const int nj = jc[c];
  double2 acc = x[idx];
  for (int i = 0; i < nj; ++i) {
    const Z zv = Zb[(long long)i * zstride + idx];
    const double2 yy = y[i * s + c];
    cfma(acc, ccast<double2>(zv), yy);
  }
  x[idx] = acc;
}

__global__ void zero_kernel(unsigned int* p, long long words) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < words) p[i] = 0u;
}

__global__ void zero_column_kernel(double2* x, long long n, int s, int col) {
  const long long node = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (node < n) x[node * s + col] = make_double2(0.0, 0.0);
}

__global__ void point_sources_kernel(const int* __restrict__ idx, const double* __restrict__ amp,
                                     int nrhs, const double2* px, const double2* py,
                                     const double2* pz, int nx, int ny, int nz, double2* b) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nrhs) return;
  const int i = idx[3 * c], j = idx[3 * c + 1], k = idx[3 * c + 2];
  const double2 S = cmul(cmul(px[2 * i + 1], py[2 * j + 1]), pz[2 * k + 1]);
  const double2 a = amp ? make_double2(amp[2 * c], amp[2 * c + 1]) : make_double2(1.0, 0.0);
  const long long n = (long long)nx * ny * nz;
  b[(long long)c * n + ((long long)k * ny + j) * nx + i] = cmul(a, S);
}

__global__ void sample_kernel(const double2* __restrict__ u, long long n, int nrhs,
                              const int* __restrict__ rec, int nrec, int nx, int ny,
                              double2* __restrict__ d) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)nrhs * nrec) return;
  const int c = (int)(idx / nrec), r = (int)(idx % nrec);
  const long long node = ((long long)rec[3 * r + 2] * ny + rec[3 * r + 1]) * nx + rec[3 * r];
  d[idx] = u[(long long)c * n + node];
}

// one thread per column, receivers in order: deterministic sums of duplicates
__global__ void spread_kernel(const double2* __restrict__ d, long long n, int nrhs,
                              const int* __restrict__ rec, int nrec, int nx, int ny,
                              double2* __restrict__ b) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nrhs) return;
  for (int r = 0; r < nrec; ++r) {
    const long long node = ((long long)rec[3 * r + 2] * ny + rec[3 * r + 1]) * nx + rec[3 * r];
    b[(long long)c * n + node] = cadd(b[(long long)c * n + node], d[(long long)c * nrec + r]);
  }
}

// g_i = -Re omega^2 q_i sum_c [ wm0_i S_i conj(mu_i) u_i
//        + sum_{j~i} 1/2 mhat_ij (conj(mu_i) u_j + conj(mu_j) u_i) ],
// mhat_ij = 1/2 (wm_t,i + wm_t,j) 1/2 (S_i + S_j)
__global__ void gradient_kernel(OpView V, const double2* __restrict__ qfac,
                                const double2* __restrict__ u, const double2* __restrict__ mu,
                                int nrhs, double* __restrict__ gout) {
  const long long n = (long long)V.nx * V.ny * V.nz;
  const long long node = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= n) return;
  const int i = (int)(node % V.nx);
  const int j = (int)((node / V.nx) % V.ny);
  const int k = (int)(node / ((long long)V.nx * V.ny));
  const double2 Si = cmul(cmul(V.px[2 * i + 1], V.py[2 * j + 1]), V.pz[2 * k + 1]);
  double2 acc = make_double2(0.0, 0.0);
  {
    double2 t = make_double2(0.0, 0.0);
    for (int c = 0; c < nrhs; ++c) cfmaconj(t, mu[(long long)c * n + node], u[(long long)c * n + node]);
    acc = cscale(cmul(Si, t), V.w7[node * 7 + 3]);
  }
  for (int ez = -1; ez <= 1; ++ez)
    for (int ey = -1; ey <= 1; ++ey)
      for (int ex = -1; ex <= 1; ++ex) {
        if (ex == 0 && ey == 0 && ez == 0) continue;
        const int qi = i + ex, qj = j + ey, qk = k + ez;
        if (qi < 0 || qi >= V.nx || qj < 0 || qj >= V.ny || qk < 0 || qk >= V.nz) continue;
        const long long nb = ((long long)qk * V.ny + qj) * V.nx + qi;
        const int t = 3 + abs(ex) + abs(ey) + abs(ez);
        const double2 Sj = cmul(cmul(V.px[2 * qi + 1], V.py[2 * qj + 1]), V.pz[2 * qk + 1]);
        const double2 mh = cscale(cadd(Si, Sj), 0.25 * (V.w7[node * 7 + t] + V.w7[nb * 7 + t]));
        double2 s2 = make_double2(0.0, 0.0);
        for (int c = 0; c < nrhs; ++c) {
          cfmaconj(s2, mu[(long long)c * n + node], u[(long long)c * n + nb]);
          cfmaconj(s2, mu[(long long)c * n + nb], u[(long long)c * n + node]);
        }
        acc = cadd(acc, cscale(cmul(mh, s2), 0.5));
      }
  const double2 r = cmul(qfac[node], acc);
  gout[node] = -V.omega * V.omega * r.x;
}

template <typename R>
__global__ void cast_kernel(const double2* __restrict__ src, C<R>* __restrict__ dst,
                            long long count) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  C<R> v;
  v.x = (R)src[i].x;
  v.y = (R)src[i].y;
  dst[i] = v;
}

__global__ void widen_kernel(const float2* __restrict__ src, double2* __restrict__ dst,
                             long long count) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float2 v = src[i];
  dst[i] = make_double2((double)v.x, (double)v.y);
}

inline unsigned blocks_for(long long work, int bs) { return (unsigned)((work + bs - 1) / bs); }
inline int group_threads(int s) {
  int G = 256 / s;
  if (G < 1) G = 1;
  return G * s;
}

}  // namespace

void launch_to_internal(const double2* src, double2* dst, long long n, int nrhs, int s, int conj,
                        hipStream_t st) {
  hipLaunchKernelGGL(to_internal_kernel, dim3(blocks_for(n * s, 256)), dim3(256), 0, st, src, dst,
                     n, nrhs, s, conj);
}
void launch_from_internal(const double2* src, double2* dst, long long n, int nrhs, int s, int conj,
                          hipStream_t st) {
  const dim3 grid((unsigned)((n + TR_NODES - 1) / TR_NODES),
                  (unsigned)((nrhs + TR_COLS - 1) / TR_COLS));
  hipLaunchKernelGGL(from_internal_kernel, grid, dim3(256), 0, st, src, dst, n, nrhs, s, conj);
}
void launch_colnorm2(const double2* x, long long n, int s, double* partial, int nblk,
                     hipStream_t st) {
  hipLaunchKernelGGL(colnorm2_kernel, dim3(nblk), dim3(group_threads(s)), 0, st, x, n, s, partial);
}
void launch_finish_norm(const double* partial, int nblk, int s, double* out, hipStream_t st) {
  hipLaunchKernelGGL(finish_norm_kernel, dim3(s), dim3(256), 0, st, partial, nblk, s, out);
}
template <typename W>
void launch_cgs_dot(const double2* V, long long vstride, int j1, const W* w, long long n, int s,
                    double2* partial, int nblk, hipStream_t st) {
  hipLaunchKernelGGL((cgs_dot_kernel<W>), dim3(nblk), dim3(group_threads(s)), 0, st, V, vstride,
                     j1, w, n, s, partial);
}
template void launch_cgs_dot<double2>(const double2*, long long, int, const double2*, long long,
                                      int, double2*, int, hipStream_t);
template void launch_cgs_dot<float2>(const double2*, long long, int, const float2*, long long,
                                     int, double2*, int, hipStream_t);
void launch_cgs_finish_dot(const double2* partial, int nblk, int j1, int s, const double* scale,
                           double2* h, double2* hs, hipStream_t st) {
  hipLaunchKernelGGL(cgs_finish_dot_kernel, dim3(j1 * s), dim3(256), 0, st, partial, nblk, j1, s,
                     scale, h, hs);
}
template <typename W>
void launch_cgs_update(const double2* V, long long vstride, int j1, const double2* hs,
                       const W* win, double2* wout, long long n, int s, double* partial, int nblk,
                       hipStream_t st) {
  hipLaunchKernelGGL((cgs_update_kernel<W>), dim3(nblk), dim3(group_threads(s)), 0, st, V,
                     vstride, j1, hs, win, wout, n, s, partial);
}
template void launch_cgs_update<double2>(const double2*, long long, int, const double2*,
                                         const double2*, double2*, long long, int, double*, int,
                                         hipStream_t);
template void launch_cgs_update<float2>(const double2*, long long, int, const double2*,
                                        const float2*, double2*, long long, int, double*, int,
                                        hipStream_t);
void launch_arnoldi_step(int j, int m, int s, const double* hnorm, const double2* h, double2* H,
                         double* cs, double2* sn, double2* g, double* scale_next, int* jc,
                         int* done, const double* bnorm, double tol, double* est,
                         hipStream_t st) {
  hipLaunchKernelGGL(arnoldi_step_kernel, dim3(blocks_for(s, 64)), dim3(64), 0, st, j, m, s, hnorm,
                     h, H, cs, sn, g, scale_next, jc, done, bnorm, tol, est);
}
void launch_cycle_init(int s, int m, const double* beta, const int* conv, double2* g,
                       double* scale0, int* jc, int* done, hipStream_t st) {
  hipLaunchKernelGGL(cycle_init_kernel, dim3(blocks_for(s, 64)), dim3(64), 0, st, s, m, beta, conv,
                     g, scale0, jc, done);
}
void launch_backsolve(int m, int s, const double2* H, const double2* g, const int* jc, double2* y,
                      hipStream_t st) {
  hipLaunchKernelGGL(backsolve_kernel, dim3(blocks_for(s, 64)), dim3(64), 0, st, m, s, H, g, jc, y);
}
template <typename Z>
void launch_update_x(const Z* Zb, long long zstride, const double2* y, const int* jc, double2* x,
                     long long n, int s, hipStream_t st) {
  hipLaunchKernelGGL((update_x_kernel<Z>), dim3(blocks_for(n * s, 256)), dim3(256), 0, st, Zb,
                     zstride, y, jc, x, n, s);
}
template void launch_update_x<float2>(const float2*, long long, const double2*, const int*,
                                      double2*, long long, int, hipStream_t);
template void launch_update_x<double2>(const double2*, long long, const double2*, const int*,
                                       double2*, long long, int, hipStream_t);

void launch_zero(void* p, size_t bytes, hipStream_t st) {
  const long long words = (long long)(bytes / 4);
  if (words == 0) return;
  hipLaunchKernelGGL(zero_kernel, dim3(blocks_for(words, 256)), dim3(256), 0, st,
                     (unsigned int*)p, words);
}
void launch_zero_column(double2* x, long long n, int s, int col, hipStream_t st) {
  hipLaunchKernelGGL(zero_column_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, x, n, s, col);
}
void launch_point_sources(const int* idx, const double* amp, int nrhs, const double2* px,
                          const double2* py, const double2* pz, int nx, int ny, int nz,
                          double2* b, hipStream_t st) {
  hipLaunchKernelGGL(point_sources_kernel, dim3(blocks_for(nrhs, 64)), dim3(64), 0, st, idx, amp,
                     nrhs, px, py, pz, nx, ny, nz, b);
}
void launch_sample(const double2* u, long long n, int nrhs, const int* rec, int nrec, int nx,
                   int ny, double2* d, hipStream_t st) {
  hipLaunchKernelGGL(sample_kernel, dim3(blocks_for((long long)nrhs * nrec, 256)), dim3(256), 0,
                     st, u, n, nrhs, rec, nrec, nx, ny, d);
}
void launch_spread(const double2* d, long long n, int nrhs, const int* rec, int nrec, int nx,
                   int ny, double2* b, hipStream_t st) {
  hipLaunchKernelGGL(spread_kernel, dim3(blocks_for(nrhs, 64)), dim3(64), 0, st, d, n, nrhs, rec,
                     nrec, nx, ny, b);
}
void launch_gradient(const OpView& op, const double2* qfac, const double2* u, const double2* mu,
                     int nrhs, double* g, hipStream_t st) {
  const long long n = (long long)op.nx * op.ny * op.nz;
  hipLaunchKernelGGL(gradient_kernel, dim3(blocks_for(n, 128)), dim3(128), 0, st, op, qfac, u, mu,
                     nrhs, g);
}
template <typename R>
void launch_cast(const double2* src, C<R>* dst, long long count, hipStream_t st) {
  hipLaunchKernelGGL((cast_kernel<R>), dim3(blocks_for(count, 256)), dim3(256), 0, st, src, dst,
                     count);
}
template void launch_cast<float>(const double2*, float2*, long long, hipStream_t);
template void launch_cast<double>(const double2*, double2*, long long, hipStream_t);
void launch_widen(const float2* src, double2* dst, long long count, hipStream_t st) {
  hipLaunchKernelGGL(widen_kernel, dim3(blocks_for(count, 256)), dim3(256), 0, st, src, dst,
                     count);
}

}  // namespace oras
