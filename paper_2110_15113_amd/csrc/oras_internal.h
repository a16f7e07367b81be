// Internal declarations of the ORAS-FGMRES Helmholtz library (gfx950).
// Shared by the host driver and the kernel translation units only.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/oras.h"

namespace oras {

// ---------------------------------------------------------------- complex --
template <typename R> struct cplx;
template <> struct cplx<float> { using type = float2; };
template <> struct cplx<double> { using type = double2; };
template <typename R> using C = typename cplx<R>::type;

template <typename R> __host__ __device__ inline C<R> mk(R a, R b) { C<R> z; z.x = a; z.y = b; return z; }
template <typename T> __host__ __device__ inline T cadd(T a, T b) { a.x += b.x; a.y += b.y; return a; }
template <typename T> __host__ __device__ inline T csub(T a, T b) { a.x -= b.x; a.y -= b.y; return a; }
template <typename T> __host__ __device__ inline T cmul(T a, T b) {
  T z; z.x = a.x * b.x - a.y * b.y; z.y = a.x * b.y + a.y * b.x; return z;
}
// Fused multiply-add by component type.  The complex updates below are written
// as explicit chains of these: left as acc += (a b - c d) the compiler may
// only fuse inside the bracket, which costs a multiply, a fused multiply-add
// and an add per component instead of two fused multiply-adds.
__host__ __device__ inline float rfma(float a, float b, float c) { return fmaf(a, b, c); }
__host__ __device__ inline double rfma(double a, double b, double c) { return fma(a, b, c); }
// acc += a * b
template <typename T> __host__ __device__ inline void cfma(T& acc, T a, T b) {
  acc.x = rfma(a.x, b.x, acc.x); acc.x = rfma(-a.y, b.y, acc.x);
  acc.y = rfma(a.x, b.y, acc.y); acc.y = rfma(a.y, b.x, acc.y);
}
// acc -= a * b
template <typename T> __host__ __device__ inline void cfms(T& acc, T a, T b) {
  acc.x = rfma(-a.x, b.x, acc.x); acc.x = rfma(a.y, b.y, acc.x);
  acc.y = rfma(-a.x, b.y, acc.y); acc.y = rfma(-a.y, b.x, acc.y);
}
// acc += conj(a) * b
template <typename T> __host__ __device__ inline void cfmaconj(T& acc, T a, T b) {
  acc.x = rfma(a.x, b.x, acc.x); acc.x = rfma(a.y, b.y, acc.x);
  acc.y = rfma(a.x, b.y, acc.y); acc.y = rfma(-a.y, b.x, acc.y);
}
template <typename T> __host__ __device__ inline T cscale(T a, double s) { a.x *= s; a.y *= s; return a; }
__host__ __device__ inline double2 cdiv(double2 a, double2 b) {
  double d = b.x * b.x + b.y * b.y;
  return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
__host__ __device__ inline double2 cinv(double2 b) {
  double d = b.x * b.x + b.y * b.y;
  return make_double2(b.x / d, -b.y / d);
}
template <typename To, typename From> __host__ __device__ inline To ccast(From a) {
  To z; z.x = a.x; z.y = a.y; return z;
}

// ------------------------------------------- FP32 products on bf16 MFMA --
// An FP32 value is split exactly into three bf16 pieces, x = x1 + x2 + x3,
// each the round-to-nearest-even of what the previous pieces leave (a 24-bit
// significand leaves at most 8 bits for the last piece).  A real product is
// then the sum of the six piece products at least 2^-16 of the leading one
// (a1 b1, a1 b2, a2 b1, a1 b3, a3 b1, a2 b2); the three left out are below
// 2^-24 |a b|, so the product carries an FP32-level error on the bf16 matrix
// instruction.
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// Two FP32 values rounded to bf16 (round to nearest even), packed: a low, b high.
__device__ inline unsigned pack_bf16(float a, float b) {
  const f32x2 v = {a, b};
  return __builtin_bit_cast(unsigned, __builtin_convertvector(v, bf16x2));
}
__device__ inline float bf16_lo(unsigned p) { return __builtin_bit_cast(float, p << 16); }
__device__ inline float bf16_hi(unsigned p) { return __builtin_bit_cast(float, p & 0xffff0000u); }
// a = a1 + a2 + a3 and b likewise, each piece word holding (a_i, b_i).
__device__ inline void split3(float a, float b, unsigned& w1, unsigned& w2, unsigned& w3) {
  w1 = pack_bf16(a, b);
  a -= bf16_lo(w1);
  b -= bf16_hi(w1);
  w2 = pack_bf16(a, b);
  a -= bf16_lo(w2);
  b -= bf16_hi(w2);
  w3 = pack_bf16(a, b);
}
__device__ inline bf16x8 as_bf16x8(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }


// ---------------------------------------------------------------- layouts --
constexpr int TILE = 32;        // factor tile edge (complex entries)
constexpr int RHS_ALIGN = 8;    // internal right-hand-side count granularity
// Column count of the plane right-hand-side buffer (blocks of 16 columns).
__host__ __device__ constexpr inline long long pad16(long long s) { return (s + 15) / 16 * 16; }
__host__ __device__ constexpr inline long long pad32(long long s) { return (s + 31) / 32 * 32; }
// Bytes of the plane right-hand-side buffer for tv_rows plane rows and s
// columns.  Complex FP32 factors take t as three bf16 pieces of each real and
// imaginary part (12 bytes per complex entry) in chunks of 32 columns;
// complex FP64 factors take t row-major in blocks of 16 columns.
inline size_t plane_rhs_bytes(int factor_prec, long long tv_rows, long long s) {
  return factor_prec == ORAS_C64 ? (size_t)(tv_rows * pad32(s)) * 12
                                 : (size_t)(tv_rows * pad16(s)) * sizeof(double2);
}

// Neighbour offset (ex, ey, ez) in {-1,0,1}^3 -> coefficient slot.
__host__ __device__ constexpr inline int eidx(int ex, int ey, int ez) {
  return (ez + 1) * 9 + (ey + 1) * 3 + (ex + 1);
}

// Operator description visible to the assembly kernels (all device memory).
struct OpView {
  int nx, ny, nz;
  double h, omega;
  const double* w7;      // (n, 7): w1 w2 w3 wm0 wmf wme wmc per node
  const double2* mt;     // (n) complex squared slowness
  const double2* px;     // PML profile on the half grid, length 2 nx + 1
  const double2* py;
  const double2* pz;
};

// One overlapping subdomain: box [lo, hi) and owned cuboid [olo, ohi).
struct SubDesc {
  int lo[3], hi[3], olo[3], ohi[3];
  int sx, sy, sz;        // box extents
  int p;                 // plane size sx*sy
  int P;                 // padded plane size (multiple of TILE)
  int nt;                // P / TILE
  int pad_;
  long long fac_off;     // complex offset of plane 0's inverse in the factor buffer
  long long lca_off;     // offset of the local coefficient array (27 * sx*sy*sz)
  long long y_off;       // offset of the local solution buffer (sz * P * s)  [in units of P*s]
  long long t_off;       // offset of the scratch plane (P*P) used while factoring
  long long tv_off;      // first plane row of the plane right-hand side (P rows)
};

// ------------------------------------------------------------- launchers --
// Assembly
void launch_assemble_global(const OpView& op, double2* coef, hipStream_t s);
// Interface condition of the local matrices (kind ORAS_IFACE_ROBIN or
// ORAS_IFACE_PML; the PML layer law uses c_ref, R0 and power).
struct IfaceView {
  int kind;
  int power;
  double c_ref, R0;
};
void launch_assemble_local(const OpView& op, const SubDesc* subs_dev, int nsub, long long max_box,
                           void* lca, int prec, const IfaceView& ifc, hipStream_t s);
void launch_fields(const double* vel, const double* q, const double* m_override, const double* wtab,
                   int tab_count, double g0, double dg, int nx, int ny, int nz, double h,
                   double omega, double* w7, double2* qfac, double2* mt, hipStream_t s,
                   int keep_weights);
void launch_pml(double2* prof, int n, int npml, double h, double omega, double c_ref, double R0,
                int power, int low, int high, hipStream_t s);
// Validity check of a model array x (n doubles, every entry must be finite and
// > 0): out[0] = maximum of the valid entries, out[1] = number of invalid
// ones.  out holds field_check_doubles() doubles (partials after the first two).
long long field_check_doubles();
void launch_field_check(const double* x, long long n, double* out, hipStream_t s);

// Node fields of the matrix-free 27-point apply in the stencil precision R:
// per node (wm_f, wm_e, wm_c, Re m~) and Im m~ (the mass weights of the
// face, edge and corner shells and the complex squared slowness; the centre
// weight is 1 - 6 wm_f - 12 wm_e - 8 wm_c).  The stiffness part needs only the
// 1D PML profiles and the three family weights, which the weight table keeps
// constant over G; the profiles enter through per-axis factor tables, nine
// complex values per node coordinate i: R(d), H(d), N(d) for d = -1, 0, +1
// with R(+-1) = 1 / s(i +- 1/2), H(+-1) = s(i +- 1/2), R(0) and H(0) the sums
// of the two, N(d) = s(i + d) (half-grid indices clamped to the profile).
template <typename R> struct R4;
template <> struct R4<float> { using type = float4; };
template <> struct R4<double> { using type = double4; };
template <typename R> struct StencilMF {
  const typename R4<R>::type* f4;
  const R* fim;
  const C<R>* fx;        // factor tables, 9 per node coordinate along each axis
  const C<R>* fy;
  const C<R>* fz;
  const int4* tiles;     // tiles (i0, j0, k0, k1), PML-free ones first (stencil_mf_tiles)
  int ntiles, nplain;
  double W1, W2, W3;     // stiffness family weights: w1 / h^2, w2 / (8 h^2), w3 / (16 h^2)
  double om2;            // omega^2
};
template <typename R>
void launch_mass_fields(const double* w7, const double2* mt, long long n,
                        typename R4<R>::type* f4, R* fim, hipStream_t st);
// The apply's tiles as (i0, j0, k0, k1) quadruples, the nplain PML-free ones
// first (every node within [lo, hi) per axis: all profile values its row
// uses are 1), then the PML tiles covering the rest of the grid.
void stencil_mf_tiles(const int lo[3], const int hi[3], int nx, int ny, int nz,
                      std::vector<int>& tiles, int& nplain);
// y = A x (or b - A x) in [n][s] layout; y is complex128, or complex64 for
// the single-precision apply without b (its values are FP32 ones either way).
template <typename R, typename Y = double2>
void launch_stencil_mf(const StencilMF<R>& op, const C<R>* x, const double2* b, Y* y, int nx,
                       int ny, int nz, int s, hipStream_t st);


// Factorisation, one plane for all subdomains.  stats (2 per subdomain plane,
// zeroed before the first plane) receives the bits of max |S_k|^2 and of
// max 1 / |pivot|^2 (non-negative doubles, whose bits order as their values).
template <typename R>
void launch_factor_plane(const SubDesc* subs_dev, int nsub, int k, int max_nt, int max_sz,
                         C<R>* fac, C<R>* tbuf, const C<R>* lca, int* status,
                         unsigned long long* stats, hipStream_t st);

// Shape of the ORAS apply: the 2 max_sz - 1 plane steps (forward k = 0..,
// then backward k = max_sz - 2..0) over the subdomain descriptors.
struct OrasPlan {
  const SubDesc* subs = nullptr;   // device
  int nsub = 0;
  int max_sz = 0;
  int max_nt = 0;
  long long max_p = 0;
};

// Tri-solve (ORAS apply).  Input v (double2, global [n][s]) times per-column scale
// (may be null) -> output z (global [n][s], precision Z).  gemm_ev (2 per step,
// or null) brackets every plane GEMM with HIP events.
template <typename R, typename Z>
void launch_oras_apply(const OrasPlan& plan, const C<R>* fac, const C<R>* lca, C<R>* ybuf,
                       C<R>* tvbuf, const double2* v, const double* scale, Z* z, int nx, int ny,
                       int s, hipStream_t st, hipEvent_t* gemm_ev = nullptr);

// Krylov helpers
void launch_to_internal(const double2* src, double2* dst, long long n, int nrhs, int s, int conj,
                        hipStream_t st);
void launch_from_internal(const double2* src, double2* dst, long long n, int nrhs, int s, int conj,
                          hipStream_t st);
void launch_colnorm2(const double2* x, long long n, int s, double* partial, int nblk, hipStream_t st);
void launch_finish_norm(const double* partial, int nblk, int s, double* out, hipStream_t st);
template <typename W>
void launch_cgs_dot(const double2* V, long long vstride, int j1, const W* w, long long n, int s,
                    double2* partial, int nblk, hipStream_t st);
void launch_cgs_finish_dot(const double2* partial, int nblk, int j1, int s, const double* scale,
                           double2* h, double2* hs, hipStream_t st);
template <typename W>
void launch_cgs_update(const double2* V, long long vstride, int j1, const double2* hs,
                       const W* win, double2* wout, long long n, int s, double* partial, int nblk,
                       hipStream_t st);
void launch_arnoldi_step(int j, int m, int s, const double* hnorm, const double2* h, double2* H,
                         double* cs, double2* sn, double2* g, double* scale_next, int* jc,
                         int* done, const double* bnorm, double tol, double* est,
                         hipStream_t st);
void launch_cycle_init(int s, int m, const double* beta, const int* conv, double2* g,
                       double* scale0, int* jc, int* done, hipStream_t st);
void launch_backsolve(int m, int s, const double2* H, const double2* g, const int* jc, double2* y,
                      hipStream_t st);
template <typename Z>
void launch_update_x(const Z* Zb, long long zstride, const double2* y, const int* jc, double2* x,
                     long long n, int s, hipStream_t st);
void launch_zero(void* p, size_t bytes, hipStream_t st);
void launch_zero_column(double2* x, long long n, int s, int col, hipStream_t st);
void launch_point_sources(const int* idx, const double* amp, int nrhs, const double2* px,
                          const double2* py, const double2* pz, int nx, int ny, int nz,
                          double2* b, hipStream_t st);
void launch_sample(const double2* u, long long n, int nrhs, const int* rec, int nrec, int nx,
                   int ny, double2* d, hipStream_t st);
void launch_spread(const double2* d, long long n, int nrhs, const int* rec, int nrec, int nx,
                   int ny, double2* b, hipStream_t st);
void launch_gradient(const OpView& op, const double2* qfac, const double2* u, const double2* mu,
                     int nrhs, double* g, hipStream_t st);
template <typename R>
void launch_cast(const double2* src, C<R>* dst, long long count, hipStream_t st);
// dst = src exactly (complex64 -> complex128)
void launch_widen(const float2* src, double2* dst, long long count, hipStream_t st);

// ------------------------------------------------- block low-rank inverses --
// Patch grid of one subdomain plane (rectangles of at most pmax x pmax nodes)
// and its rows of the operand buffer: the plane right-hand side in
// patch-major order (each patch's rows padded to a multiple of 8, padding
// rows zero), then the projection rows T.
struct BlrSub {
  long long bt_off;      // first operand-buffer row of the subdomain
  int npx, npy;
  int ptab;              // offset in the list array of the patches' first t rows
  int pad_;
};
// One patch block (I, J) of one plane inverse: where compression writes it.
struct BlrBlock {
  int sub, k, I, J;
  int rank;              // planned rank (-1: stored dense)
  int e_koff;            // first K column of the block in the expansion operand of patch I
  int p_mpad;            // row stride of the projection operand of patch J
  int p_row;             // first row of the block's V in that operand
  long long e_off;       // complex offset of the expansion operand of patch I
  long long p_off;       // complex offset of the projection operand of patch J (-1: none)
};
// One wave's work in a segment GEMM: rows of the output of one patch.
// Operand rows come in segments of consecutive operand-buffer rows whose
// lengths are multiples of 8.
struct BlrItem {
  int sub;               // -1: padding (no work)
  int patch;
  int rows;              // valid output rows
  int mpad;              // row stride of the operand storage ([k / 4][row][k % 4])
  int K;                 // operand columns, a multiple of 8
  int row0;              // first operand row of this item
  int brow;              // projection: operand-buffer row (from bt_off) of the patch's t rows
  int nseg;              // expansion: segments {k0, row, length, 0} at list_off
  long long a_off;       // complex offset of the operand storage
  long long list_off;    // projection: 32 destination rows; expansion: the segments
};
struct BlrApply {
  const SubDesc* subs;
  const BlrSub* bsubs;
  const BlrItem* items;
  const int* lists;
  int nsub, max_sz;
  long long max_p;
  // per plane k: [first, count) of the projection and expansion items
  std::vector<int> p_first, p_count, e_first, e_count;
};
constexpr int BLR_PMAX = 8;     // largest patch edge (64-node patches)

template <typename R>
void launch_blr_plane_max(const SubDesc* subs, int nsub, int max_sz, const C<R>* fac,
                          double* smax, hipStream_t st);
// rank_out (pass without astore) or the compressed operands (pass with astore;
// err[0] is set when a block's rank differs from the planned one)
template <typename R>
void launch_blr_compress(const SubDesc* subs, const BlrSub* bsubs, const BlrBlock* blocks,
                         long long nblocks, const C<R>* fac, const double* smax, int max_sz,
                         double eps, int* rank_out, C<R>* astore, int* err, hipStream_t st);
template <typename R, typename Z>
void launch_oras_apply_blr(const BlrApply& pl, const C<R>* astore, const C<R>* lca, C<R>* ybuf,
                           C<R>* bt, const double2* v, const double* scale, Z* z, int nx, int ny,
                           int s, hipStream_t st, hipEvent_t* gemm_ev = nullptr);

// Stencil-weight part of the gradient (weights following m): g -= sum_k
// dw_k/dm Re H_k.  scratch holds weight_grad_scratch(nx, ny, nz) doubles.
long long weight_grad_scratch(int nx, int ny, int nz);
void launch_weight_gradient(const OpView& op, const double2* qfac, const double* wtab,
                            int tab_count, double g0, double dg, const double2* u,
                            const double2* mu, int nrhs, double* scratch, double* g,
                            hipStream_t st);

// ------------------------------------------------- shared by entry points --
// (defined in oras_api.cpp, which owns the context layout)
oras_status check_apply_A(oras_ctx c, const void* x_dev, const void* y_dev, int nrhs, int prec);
// staging bytes of apply_A_staged: x and y in the internal layout (complex128)
// plus, for prec ORAS_C64, x rounded to complex64
size_t apply_A_scratch_bytes(oras_ctx c, int nrhs, int prec);
oras_status apply_A_staged(oras_ctx c, const void* x_dev, void* y_dev, int nrhs, int prec,
                           double2* xin, double2* yout, float2* x32);
oras_status set_error(oras_ctx c, oras_status st, const char* msg);
int ctx_device(oras_ctx c);
// Records the address of `device`'s copy of the no-alloc scratch array
// (noalloc.hip); the device must be current.  Called once per context
// creation, does the lookup once per device.
oras_status noalloc_init(int device);

}  // namespace oras
