// Internal declarations shared by the HIP sources of the ltd library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <algorithm>

namespace ltd {

// ----------------------------------------------------------------------------
// Complex helpers (interleaved re/im in double2 / float2)
// ----------------------------------------------------------------------------
__host__ __device__ inline double2 cmake(double r, double i) { return make_double2(r, i); }
__host__ __device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline double2 cmulc(double2 a, double2 b) {  // conj(a) * b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__host__ __device__ inline double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__host__ __device__ inline double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__host__ __device__ inline double2 cfma(double2 a, double2 b, double2 c) {  // a*b + c
  return make_double2(fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y)));
}
__host__ __device__ inline float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__host__ __device__ inline float2 cconj(float2 a) { return make_float2(a.x, -a.y); }

// Complex element types of the transforms: double2 (FP64) and float2 (FP32).
template <class T>
struct CT;
template <>
struct CT<double2> {
  using R = double;
  __host__ __device__ static double2 mk(double x, double y) { return make_double2(x, y); }
  __host__ __device__ static double2 from(double2 a) { return a; }
};
template <>
struct CT<float2> {
  using R = float;
  __host__ __device__ static float2 mk(float x, float y) { return make_float2(x, y); }
  __host__ __device__ static float2 from(double2 a) { return make_float2((float)a.x, (float)a.y); }
};
__host__ __device__ inline double2 to_d2(double2 a) { return a; }
__host__ __device__ inline double2 to_d2(float2 a) { return make_double2(a.x, a.y); }

// ----------------------------------------------------------------------------
// GEMM: C = alpha op(A) op(B) + beta C, complex128, column-major.
// ----------------------------------------------------------------------------
enum Op { OP_N = 0, OP_C = 1 };

struct ZProb {
  const double2 *A;
  const double2 *B;
  double2 *C;
  // optional two-segment K for op(B) = N: rows k < kseg of B come from B, rows
  // k >= kseg from B2 (row k - kseg); kseg = 0 disables
  const double2 *B2;
  int kseg;
  long long sA, sB, sC;  // batch strides (elements)
  int lda, ldb, ldc;
  int m, n, k, batch;
  double2 alpha, beta;
  // planner-filled
  int tiles_m, tiles_n, ksplit, kchunk;  // kchunk: K per split, multiple of the K tile
  int bm;                                // output tile rows (64 or 32), the same for a whole launch
  int tile_begin;                        // first logical tile of this problem
  int rtile_begin;                       // first output tile (reduction pass)
  long long part_off;                    // offset (tiles) into the split-K partial buffer
  // launch-wide (the same in every problem): the output tiles of the launch when
  // its logical tiles run K-chunk-major (every problem split by the same factor:
  // the tiles of one K chunk of all problems are adjacent), else 0
  int kmajor;
};

constexpr int GEMM_MAXP = 8;  // problems passed by value in one launch

struct ZBatch {
  ZProb p[GEMM_MAXP];
  int nprob;
  int total_tiles;
};

// Plans (tiles, split-K) a batch in place; returns the partial-buffer size (bytes).
// `target_blocks` is the launch size below which K is split.
// Split-K partial tiles never exceed `max_part_tiles` (64x64 complex each).
size_t gemm_plan(ZProb *probs, int nprob, int *total_tiles, int target_blocks = 512,
                 long long max_part_tiles = 2048);
// Launches a planned batch held by value (nprob <= GEMM_MAXP).
hipError_t gemm_launch(int opa, int opb, const ZBatch &b, double2 *partials, hipStream_t s);
// Launches a planned batch whose problem table lives in device memory (any size);
// `host` is the same table on the host (for the reduction pass).
// n_limit > 0 caps every problem's column count (tiles beyond it exit at once).
// parts: 1 the product kernel, 2 the split-K reduction (when K is split), 3 both.
hipError_t gemm_launch_table(int opa, int opb, const ZProb *dev_table, const ZProb *host, int nprob,
                             int total_tiles, double2 *partials, int n_limit, hipStream_t s, int parts = 3);

// The same GEMMs on complex64 operands (ZProb pointers holding float2 data) with
// FP32 matrix cores, FP32 sums per K tile of 16 and FP64 sums across tiles and
// splits, op(B) = B.  Planned by gemm_plan like the FP64 ones.  C in complex128,
// or (out32, unsplit problems only) in complex64.
hipError_t cgemm32_launch(int opa, const ZBatch &b, double2 *partials, hipStream_t s, bool out32 = false);
hipError_t cgemm32_launch_table(int opa, const ZProb *dev_table, const ZProb *host, int nprob, int total_tiles,
                                double2 *partials, hipStream_t s, int parts = 3, bool out32 = false);

// ----------------------------------------------------------------------------
// Interstitial FFT pipeline.
// ----------------------------------------------------------------------------
constexpr int FFT_MAXST = 8;
constexpr int FFT_MAXLEN = 192;

struct FftPlan {
  int L;
  int nst;
  int radix[FFT_MAXST];
};

struct Grid {
  int n1, n2, n3;
  int bx, by, bz;  // box half-widths |g_i| <= b_i
  int nbx, nby, nbz;
  FftPlan p1, p2, p3;
  const double2 *tw1, *tw2, *tw3;  // device twiddles exp(-2 pi i m / L)
  const double *theta;             // [N]
  int d1, d2;                      // grid of the sphere tables' positions y * d1 + x
};

// Block-wide staging of e < n: store(e, load(e)), each thread issuing eight
// loads (at clamped, always valid indices) before it stores their values, so
// that the loads are in flight together.
template <class T, class LD, class ST>
__device__ __forceinline__ void stage8(int n, LD load, ST store) {
  const int nt = blockDim.x;
  for (int e0 = threadIdx.x; e0 < n; e0 += 8 * nt) {
    T r[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = e0 + q * nt;
      r[q] = load(e < n ? e : n - 1);
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = e0 + q * nt;
      if (e < n) store(e, r[q]);
    }
  }
}

// Per-k sphere tables (device).
struct KSphere {
  const double *gk;       // [n_g][3]
  const int *plane_ptr;   // [nbz+1] CSR over kz planes
  const int *pts_g;       // [n_g] G index, sorted by plane
  const int *pts_xy;      // [n_g] position y*N1 + x of the point in its plane
  const int *plane_x;     // [2 nbz] box-x range [lo, hi) of each plane's points (lo = hi: none)
  int n_g;
};

enum FftMode { FFT_MODE_V = 0, FFT_MODE_HS = 1, FFT_MODE_TVPS = 2 };

// Output descriptor of the forward plane pass (one per k).
struct FwdOut {
  double2 *o0;  // MODE_V: Y;  MODE_HS: HC;  MODE_TVPS: T
  float2 *o0f;  // rebuild read-out: when set, Y goes here in complex64 instead of to o0
  double2 *o1;  // MODE_HS: SC;  MODE_TVPS: V
  double2 *o2;  // MODE_TVPS: P
  double2 *o3;  // MODE_TVPS: S
  int ld0, ld1, ld2, ld3;
};

// Input descriptor of the inverse plane pass (one per k): plane-wave block of C.
struct InvIn {
  const double2 *c;
  int ldc;
};

constexpr int FFT_MAXK = 16;  // k-points handled by one batched FFT launch

struct FftKArgs {
  KSphere sph[FFT_MAXK];
  InvIn in[FFT_MAXK];
  FwdOut out[FFT_MAXK];
  double2 *slab_in[FFT_MAXK];   // per k base of the input slabs
  double2 *slab_out[FFT_MAXK];  // per k base of the output slabs
};

// slab layout per k: [field][col][pz][y][x]; field stride = ncols * nbz * N1 * N2.
// Box route of the apply (square 72- or 64-point planes with the register x/z
// kernel, box within the exact-grid bound): fft_ap_inverse_y writes the y images
// of nfields input fields (ka.sph[0], ka.in[0] -> ka.slab_out[0], field stride
// ncols * nbz * N2 * nbx); the rebuild's x/z kernel (fft_rb_step part 0, one
// pseudo k-point per field pass) and y kernel (part 1, sphere order) follow;
// fft_ap_combine forms the mode's outputs from the five (MODE_V: one) fields.
bool fft_ap_box_ok(const Grid &g);
hipError_t fft_ap_inverse_y(const Grid &g, const FftKArgs &ka, int ncols, int nfields, hipStream_t s);
hipError_t fft_ap_combine(const FwdOut &fo, const KSphere &sp, const double2 *ys, int ncols, int mode, double alpha_a,
                          double beta_a, hipStream_t s);
hipError_t fft_inverse_planes(const Grid &g, const FftKArgs &ka, int nk, int ncols, int nfields,
                              hipStream_t s);
hipError_t fft_lines(const Grid &g, const FftKArgs &ka, int nk, int ncols, int mode,
                     const double *v_r, hipStream_t s);
hipError_t fft_forward_planes(const Grid &g, const FftKArgs &ka, int nk, int ncols, int mode,
                              double alpha_a, double beta_a, hipStream_t s);

bool fft_plan_length(int L, FftPlan *p);
size_t fft_plane_lds_bytes(const Grid &g);
void fft_init_attrs();  // LDS limits of the FFT kernels (call outside graph capture)
// Per-step rebuild path: the cached grid image is c[kz][y][kx] per column
// (fft_rb_slab_values per column); fft_rb_cache builds it from sphere
// coefficients (ka.in -> ka.slab_out); fft_rb_step part 0 maps slab_in -> slab_out
// through the x/z transforms and the Theta V product, part 1 reads slab_in out to
// the sphere (ka.out[k].o0, row i = sphere-table point i, i.e. G index pts_g[i]).
size_t fft_rb_slab_values(const Grid &g);
// fp32: the cache and step slabs hold float2 (the FP32 residual); thv is then
// float, else double; Y is written in FP64 either way.
hipError_t fft_rb_cache(const Grid &g, const FftKArgs &ka, int nk, int ncols, hipStream_t s, bool fp32);
// variant: launch shape of the part-0 kernel, 0 .. fft_rb_variants(g, fp32) - 1:
// the first three are shapes of one two-factor kernel (the same arithmetic per
// value, bit-identical results); for complex64 slabs on 64-point grids a fourth
// is the register-resident kernel (the same transforms, another summation order).
hipError_t fft_rb_step(const Grid &g, const FftKArgs &ka, int nk, int ncols, const void *thv, hipStream_t s,
                       int part, bool fp32, int variant);
int fft_rb_variants(const Grid &g, bool fp32);
// Theta V of a step in the layout fft_rb_step part 0 reads (ngrid doubles).
// v is read at v + (*step) * stride when step is not NULL; vref != NULL gives
// Theta (v - vref); fp32: out is float, else double.
hipError_t fft_rb_thv(const Grid &g, const double *theta, const double *v, const int *step, long long stride,
                      void *out, const double *vref, bool fp32, hipStream_t s);
// Rebuild length of one axis of length n with box half-width b: the smallest
// length with a register path that is >= 4 b + 1 (every difference of two box
// frequencies is then distinct modulo it) and <= n; n itself otherwise.
int fft_rb_length(int n, int b);
// True when fft_rb_step has a register path for this grid (x and z lengths).
bool fft_rb_fast(const Grid &g);
// W on the rebuild grid gr from Theta V on the original grid (n1, n2, n3):
// W = IDFT_gr(keep |q_d| <= 2 b_d (DFT(Theta V))), one real matrix per axis,
// M_d[j'][j] = (1/n_d) sum_{|q| <= 2 b_d} exp(2 pi i q (j'/n'_d - j/n_d)), given by
// its table tab_d[m] = M at j'/n'_d - j/n_d = m / L_d (L_d = fft_rb_table_len);
// passes x, y, z, written in the layout fft_rb_step part 0 reads.
// t1: n3 * n2 * gr.n1 doubles, t2: n3 * gr.n2 * gr.n1 doubles.
int fft_rb_table_len(int n, int np);
// MFMA fragments of the synthesis axis matrix (n original points, np rebuild
// points) from its Dirichlet table: fft_rb_frag_len(n, np) doubles, host side.
int fft_rb_frag_len(int n, int np);
void fft_rb_frag(int n, int np, const double *tab, double *mf);
// mf_d: the fragments of M_d (device), used where n_d is 16, 64, 72 or 96; the
// tables otherwise.  sub != NULL: out = W - sub (same layout); fp32: out is
// float, else double.  plain: out in grid order [z'][y'][x'] instead of the
// order of the x/z rebuild kernel.
hipError_t fft_rb_synth(const Grid &gr, int n1, int n2, int n3, const double *th, const double *v,
                        const int *step, long long stride, const double *tab1, const double *tab2,
                        const double *tab3, const double *mf1, const double *mf2, const double *mf3, double *t1,
                        double *t2, void *out, const double *sub, bool fp32, hipStream_t s, bool plain = false);
size_t fft_line_lds_bytes(const Grid &g);

// ----------------------------------------------------------------------------
// Interstitial matrix-matrix route (dense plane-wave blocks).
// ----------------------------------------------------------------------------
// Fourier coefficients f~(q) = (1/N) sum_j f_j exp(-2 pi i q.j/N) of f = th v (th
// alone when v is NULL; v read at v + (*step) stride when step is set) in the box
// |q_d| <= 2 b_d, layout [qz][qy][qx] (mm_box_values complex); scratch:
// mm_box_scratch complex values; twiddles g.tw1..3.
size_t mm_box_values(const Grid &g);
size_t mm_box_scratch(const Grid &g);
hipError_t mm_box_coefficients(const Grid &g, const double *th, const double *v, const int *step, long long stride,
                               double2 *scratch, double2 *out, hipStream_t s);
// Dense ng x ng block (ld) of operator `which` (0 S, 1 T, 2 V, 3 P_z) at the G
// vectors gint/gk (k-point's natural order), rows and columns in the order idx
// (NULL: natural); ft = Theta~ box, fv = (Theta V)~ box.
hipError_t mm_dense(int which, const Grid &g, const int *gint, const double *gk, const int *idx, int ng,
                    const double2 *ft, const double2 *fv, double2 *out, long long ld, hipStream_t s);

}  // namespace ltd
