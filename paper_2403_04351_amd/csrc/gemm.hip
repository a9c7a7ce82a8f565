// Complex FP64 GEMM on the CDNA4 matrix cores.
//
// C = alpha op(A) op(B) + beta C with complex128 operands, column-major, as a
// grouped launch over independent problems (each optionally strided-batched)
// and an optional split of the K dimension whose partial tiles are summed in a
// fixed order by a second pass (deterministic, no atomics).
//
// Work decomposition: MB x 64 output tiles (MB = 64 or 32, chosen per launch by
// the planner), 256 threads = 4 wavefronts in a 2x2 arrangement, each
// wavefront owning an (MB/2) x 32 block of 16x16 MFMA blocks.
// A complex multiply-add is three real v_mfma_f64_16x16x4_f64 (the Gauss form
// below).  Operand tiles (64 x 16 complex)
// are staged through LDS as separate real and imaginary planes, double
// buffered, with the conjugation of op = C folded into the staging store.
// Logical tiles are remapped so that each XCD (blocks are dealt round-robin
// to the 8 XCDs) runs a contiguous range of them: tiles that share an operand
// panel share an L2.
#include "common.h"

namespace ltd {

typedef double d4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int BM = 64, BN = 64, BK = 16, NT = 256, LP = 2;  // LP: LDS row padding (doubles)
// split-K partial tiles keep a BM x BN stride whatever the tile height

template <int Q>
struct FragN {
  double2 v[Q];
};
using Frag = FragN<4>;

__device__ inline int xcd_logical(int b, int g) {
  const int q = g / 8, rem = g % 8, x = b % 8, r = b / 8;
  return (x < rem) ? x * (q + 1) + r : rem * (q + 1) + (x - rem) * q + r;
}

// Problem and tile of a logical tile.  Problem-major order: the tiles of each
// problem are contiguous (tile rows fastest, then tile columns, batch entries,
// K chunks).  K-major order (kmajor > 0, every problem split by the same factor):
// logical = ks * kmajor + the output tile's index over all problems, so the
// problems' tiles of one K chunk are adjacent and land on one XCD, where they
// share the operand panels of that chunk in L2 (the blocks of a Hermitian
// block-row product read the same columns of both operands).
struct TileAt {
  int pi, tm, tn, bi, ks;
};
__device__ inline TileAt tile_at(const ZProb *probs, int nprob, int logical) {
  TileAt r{};
  const int kmt = probs[0].kmajor;
  int t;
  if (kmt > 0) {
    const int q = logical % kmt;
    r.ks = logical / kmt;
    while (r.pi + 1 < nprob && probs[r.pi + 1].rtile_begin <= q) ++r.pi;
    t = q - probs[r.pi].rtile_begin;
  } else {
    while (r.pi + 1 < nprob && probs[r.pi + 1].tile_begin <= logical) ++r.pi;
    t = logical - probs[r.pi].tile_begin;
  }
  const ZProb &P = probs[r.pi];
  r.tm = t % P.tiles_m;
  t /= P.tiles_m;
  r.tn = t % P.tiles_n;
  t /= P.tiles_n;
  r.bi = t % P.batch;
  if (kmt == 0) r.ks = t / P.batch;
  return r;
}

// Global-memory operand pointer (address space 1: global loads, not flat ones).
typedef double d2v __attribute__((ext_vector_type(2)));
typedef const d2v __attribute__((address_space(1))) *gptr;
__device__ inline double2 ldg(gptr p) {
  const d2v v = *p;
  return make_double2(v.x, v.y);
}

// Per-block copy of the problem fields the K loop uses (registers, not the table).
struct Ops {
  gptr A, B, B2;
  int lda, ldb, m, nlim, kseg, kend;
};

// Operand loads at clamped (in-bounds) indices, zeroed by value outside the
// problem: no branch around a load, so the loads of a tile are all in flight
// together.
// A tile MB x BK: QA = MB / 16 values per thread
template <int OPA, int MB>
__device__ inline void load_a(const Ops &o, int m0, int k0, int t, FragN<MB / 16> &f) {
  constexpr int QA = MB / 16;
  if (OPA == OP_N) {  // A is m x k: tile column kk is contiguous in i
    const int kk = t >> 4, i = (t & 15) * QA;
    const int kg = k0 + kk;
    const int kc = kg < o.kend ? kg : o.kend - 1;
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int ig = m0 + i + q;
      const double2 v = ldg(o.A + (long long)(ig < o.m ? ig : o.m - 1) + (long long)kc * o.lda);
      f.v[q] = (ig < o.m && kg < o.kend) ? v : make_double2(0.0, 0.0);
    }
  } else {  // A is k x m, op = conj-transpose: tile row i is contiguous in kk
    constexpr int TPR = NT / MB;  // threads per tile row
    const int i = t / TPR, kk = (t % TPR) * QA;
    const int ig = m0 + i;
    const int ic = ig < o.m ? ig : o.m - 1;
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int kg = k0 + kk + q;
      const double2 v = ldg(o.A + (long long)(kg < o.kend ? kg : o.kend - 1) + (long long)ic * o.lda);
      f.v[q] = (ig < o.m && kg < o.kend) ? v : make_double2(0.0, 0.0);
    }
  }
}

template <int OPB>
__device__ inline void load_b(const Ops &o, int n0, int k0, int t, Frag &f) {
  if (OPB == OP_N) {  // B is k x n: tile column j is contiguous in kk
    const int j = t >> 2, kk = (t & 3) * 4;
    const int jg = n0 + j;
    const int jc = jg < o.nlim ? jg : o.nlim - 1;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int kg = k0 + kk + q;
      const int kc = kg < o.kend ? kg : o.kend - 1;
      const gptr src = (o.kseg > 0 && kc >= o.kseg) ? o.B2 + (kc - o.kseg) : o.B + kc;
      const double2 v = ldg(src + (long long)jc * o.ldb);
      f.v[q] = (jg < o.nlim && kg < o.kend) ? v : make_double2(0.0, 0.0);
    }
  } else {  // B is n x k, op = conj-transpose: tile row kk is contiguous in j
    const int kk = t >> 4, j = (t & 15) * 4;
    const int kg = k0 + kk;
    const int kc = kg < o.kend ? kg : o.kend - 1;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int jg = n0 + j + q;
      const double2 v = ldg(o.B + (long long)(jg < o.nlim ? jg : o.nlim - 1) + (long long)kc * o.ldb);
      f.v[q] = (jg < o.nlim && kg < o.kend) ? v : make_double2(0.0, 0.0);
    }
  }
}

template <int OPA, int MB>
__device__ inline void store_a(double (*As)[BK][MB + LP], int t, const FragN<MB / 16> &f) {
  constexpr int QA = MB / 16;
  const double sg = (OPA == OP_C) ? -1.0 : 1.0;
  if (OPA == OP_N) {
    const int kk = t >> 4, i = (t & 15) * QA;
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      As[0][kk][i + q] = f.v[q].x;
      As[1][kk][i + q] = f.v[q].y;
    }
  } else {
    constexpr int TPR = NT / MB;
    const int i = t / TPR, kk = (t % TPR) * QA;
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      As[0][kk + q][i] = f.v[q].x;
      As[1][kk + q][i] = sg * f.v[q].y;
    }
  }
}

template <int OPB>
__device__ inline void store_b(double (*Bs)[BK][BN + LP], int t, const Frag &f) {
  const double sg = (OPB == OP_C) ? -1.0 : 1.0;
  if (OPB == OP_N) {
    const int j = t >> 2, kk = (t & 3) * 4;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      Bs[0][kk + q][j] = f.v[q].x;
      Bs[1][kk + q][j] = f.v[q].y;
    }
  } else {
    const int kk = t >> 4, j = (t & 15) * 4;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      Bs[0][kk][j + q] = f.v[q].x;
      Bs[1][kk][j + q] = sg * f.v[q].y;
    }
  }
}

// Complex products by the three-multiplication (Gauss) form: for a = ar + i ai,
// b = br + i bi, t1 = ar br, t2 = ai bi, t3 = (ar + ai)(br + bi), and
// ab = (t1 - t2) + i (t3 - t1 - t2).  Each 16x16 output block keeps t1, t2, t3
// as three MFMA accumulators summed over K, so a complex multiply-add costs
// three real MFMAs instead of four; the sums ar + ai, br + bi are formed after
// the LDS reads.
template <int OPA, int OPB, bool TABLE, int MB>
__global__ __launch_bounds__(NT) void zgemm_kernel(const ZBatch batch, const ZProb *__restrict__ table,
                                                   int nprob, double2 *__restrict__ partials, int n_limit) {
  constexpr int AW = MB / 32;  // 16-row MFMA blocks per wavefront
  __shared__ double As[2][2][BK][MB + LP];
  __shared__ double Bs[2][2][BK][BN + LP];

  const ZProb *probs = TABLE ? table : batch.p;
  const TileAt at = tile_at(probs, nprob, xcd_logical(blockIdx.x, gridDim.x));
  const ZProb &P = probs[at.pi];
  const int tm = at.tm, tn = at.tn, bi = at.bi, ks = at.ks;

  const int m0 = tm * MB, n0 = tn * BN;
  Ops o;
  o.nlim = (n_limit > 0 && n_limit < P.n) ? n_limit : P.n;
  if (n0 >= o.nlim) return;  // whole block: columns beyond the limit
  o.A = (gptr)(const void *)(P.A + (long long)bi * P.sA);
  o.B = (gptr)(const void *)(P.B + (long long)bi * P.sB);
  o.B2 = (gptr)(const void *)(P.B2 ? P.B2 + (long long)bi * P.sB : P.B);
  o.lda = P.lda;
  o.ldb = P.ldb;
  o.m = P.m;
  o.kseg = P.B2 ? P.kseg : 0;
  const int kbeg = ks * P.kchunk;
  o.kend = min(P.k, kbeg + P.kchunk);
  const int nkt = (o.kend > kbeg) ? (o.kend - kbeg + BK - 1) / BK : 0;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;

  d4 t1[AW][2], t2[AW][2], t3[AW][2];
#pragma unroll
  for (int a = 0; a < AW; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      t1[a][b] = d4{0.0, 0.0, 0.0, 0.0};
      t2[a][b] = d4{0.0, 0.0, 0.0, 0.0};
      t3[a][b] = d4{0.0, 0.0, 0.0, 0.0};
    }

  FragN<MB / 16> fa;
  Frag fb;
  if (nkt > 0) {
    load_a<OPA, MB>(o, m0, kbeg, tid, fa);
    load_b<OPB>(o, n0, kbeg, tid, fb);
    store_a<OPA, MB>(As[0], tid, fa);
    store_b<OPB>(Bs[0], tid, fb);
  }
  __syncthreads();

  for (int kt = 0; kt < nkt; ++kt) {
    const int cur = kt & 1;
    // next tile's loads (clamped: the last iteration reloads the last tile, unused)
    const int k0 = kbeg + (kt + 1 < nkt ? kt + 1 : kt) * BK;
    load_a<OPA, MB>(o, m0, k0, tid, fa);
    load_b<OPB>(o, n0, k0, tid, fb);
    __builtin_amdgcn_sched_barrier(0);  // the loads issue before the MFMAs of this tile
#pragma unroll
    for (int kq = 0; kq < BK; kq += 4) {
      const int kk = kq + (lane >> 4);
      double ar[AW], ai[AW], as[AW], br[2], bi2[2], bs[2];
#pragma unroll
      for (int a = 0; a < AW; ++a) {
        const int i = wm * (MB / 2) + a * 16 + (lane & 15);
        ar[a] = As[cur][0][kk][i];
        ai[a] = As[cur][1][kk][i];
        as[a] = ar[a] + ai[a];
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int j = wn * 32 + b * 16 + (lane & 15);
        br[b] = Bs[cur][0][kk][j];
        bi2[b] = Bs[cur][1][kk][j];
        bs[b] = br[b] + bi2[b];
      }
#pragma unroll
      for (int a = 0; a < AW; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) t1[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[a], br[b], t1[a][b], 0, 0, 0);
#pragma unroll
      for (int a = 0; a < AW; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) t2[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[a], bi2[b], t2[a][b], 0, 0, 0);
#pragma unroll
      for (int a = 0; a < AW; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) t3[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(as[a], bs[b], t3[a][b], 0, 0, 0);
    }
    if (kt + 1 < nkt) {
      store_a<OPA, MB>(As[cur ^ 1], tid, fa);
      store_b<OPB>(Bs[cur ^ 1], tid, fb);
    }
    __syncthreads();
  }

  // Output element of accumulator register r of v_mfma_f64_16x16x4f64: row 4*r + lane/16,
  // column lane%16 (measured; the FP32 16x16 variant differs).
  const auto acc_of = [&](int a, int b, int r) {
    return make_double2(t1[a][b][r] - t2[a][b][r], t3[a][b][r] - t1[a][b][r] - t2[a][b][r]);
  };
  if (P.ksplit == 1) {
    double2 *C = P.C + (long long)bi * P.sC;
    const bool rd = (P.beta.x != 0.0 || P.beta.y != 0.0);
#pragma unroll
    for (int a = 0; a < AW; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = m0 + wm * (MB / 2) + a * 16 + 4 * r + (lane >> 4);
          const int j = n0 + wn * 32 + b * 16 + (lane & 15);
          if (i < P.m && j < o.nlim) {
            double2 v = cmul(P.alpha, acc_of(a, b, r));
            double2 *dst = C + (long long)i + (long long)j * P.ldc;
            if (rd) v = cfma(P.beta, *dst, v);
            *dst = v;
          }
        }
  } else {
    const long long tile_lin = ((long long)bi * P.tiles_n + tn) * P.tiles_m + tm;
    double2 *dst = partials + (P.part_off + tile_lin * P.ksplit + ks) * (long long)(BM * BN);
#pragma unroll
    for (int a = 0; a < AW; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int il = wm * (MB / 2) + a * 16 + 4 * r + (lane >> 4);
          const int jl = wn * 32 + b * 16 + (lane & 15);
          dst[jl * MB + il] = acc_of(a, b, r);
        }
  }
}

// Sums the split-K partials of every output tile in a fixed order, then
// C = alpha * sum + beta * C.  One thread per output element: a block covers
// RED_T consecutive elements of one tile (RED_T x 16 bytes read per split, one
// run), each thread adding splits 0, 1, ..., ksplit - 1 in order with eight
// loads in flight.
constexpr int RED_T = 256;

template <bool TABLE>
__global__ __launch_bounds__(RED_T) void zgemm_reduce(const ZBatch batch, const ZProb *__restrict__ table,
                                                      int nprob, const double2 *__restrict__ partials, int n_limit) {
  const ZProb *probs = TABLE ? table : batch.p;
  const int per_tile = (BM * BN) / RED_T;  // blocks per tile
  const int rt = blockIdx.x / per_tile;
  const int sub = blockIdx.x % per_tile;
  int pi = 0;
  while (pi + 1 < nprob && probs[pi + 1].rtile_begin <= rt) ++pi;
  const ZProb &P = probs[pi];
  if (P.ksplit == 1) return;
  const int tl = rt - P.rtile_begin;
  const int tm = tl % P.tiles_m;
  const int tn = (tl / P.tiles_m) % P.tiles_n;
  const int bi = tl / (P.tiles_m * P.tiles_n);
  const int e = sub * RED_T + threadIdx.x;
  const int mb = P.bm;
  if (e >= mb * BN) return;  // past a tile of mb < BM rows
  const int il = e % mb, jl = e / mb;
  const int i = tm * mb + il, j = tn * BN + jl;
  const int nlim = (n_limit > 0 && n_limit < P.n) ? n_limit : P.n;
  if (i >= P.m || j >= nlim) return;
  const double2 *src = partials + (P.part_off + (long long)tl * P.ksplit) * (long long)(BM * BN) + e;
  const int ks = P.ksplit;
  double2 acc = make_double2(0.0, 0.0);
  for (int q0 = 0; q0 < ks; q0 += 8) {
    double2 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = src[(long long)(q0 + u < ks ? q0 + u : ks - 1) * BM * BN];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (q0 + u < ks) acc = cadd(acc, v[u]);
  }
  double2 *C = P.C + (long long)bi * P.sC + (long long)i + (long long)j * P.ldc;
  double2 v = cmul(P.alpha, acc);
  if (P.beta.x != 0.0 || P.beta.y != 0.0) v = cfma(P.beta, *C, v);
  *C = v;
}

// ---------------------------------------------------------------------------
// Complex GEMM on complex64 operands with FP32 matrix cores (the mixed-precision
// residual rebuild): C = alpha op(A) B + beta C, op(A) = A or A^H, A and B
// complex64 column-major (the ZProb pointers hold float2 data), C complex128.
// Each K tile of BK = 16 is accumulated in FP32 by v_mfma_f32_16x16x4f32 (four
// real MFMAs per complex multiply-add: re += ar br - ai bi, im += ar bi + ai br),
// and the tiles' sums are added in FP64 registers, so the rounding of a long K
// stays that of one 16-term FP32 sum per tile; split-K partial tiles are written
// in FP64 and reduced in a fixed order by zgemm_reduce (deterministic).  Same
// tiling, planner and XCD remap as zgemm_kernel.
// ---------------------------------------------------------------------------
typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef const f2v __attribute__((address_space(1))) *gptr32;
__device__ inline float2 ldg32(gptr32 p) {
  const f2v v = *p;
  return make_float2(v.x, v.y);
}

// TO: element type of C (double2; float2 only for unsplit problems, whose C
// pointer then holds float2 data).
template <int OPA, bool TABLE, int MB, class TO>
__global__ __launch_bounds__(NT) void cgemm32_kernel(const ZBatch batch, const ZProb *__restrict__ table, int nprob,
                                                     double2 *__restrict__ partials) {
  constexpr int AW = MB / 32;
  constexpr int QA = MB / 16;
  __shared__ float As[2][2][BK][MB + 4];
  __shared__ float Bs[2][2][BK][BN + 4];
  const ZProb *probs = TABLE ? table : batch.p;
  const TileAt at = tile_at(probs, nprob, xcd_logical(blockIdx.x, gridDim.x));
  const ZProb &P = probs[at.pi];
  const int tm = at.tm, tn = at.tn, bi = at.bi, ks = at.ks;
  const int m0 = tm * MB, n0 = tn * BN;
  const gptr32 A = (gptr32)(const void *)(reinterpret_cast<const float2 *>(P.A) + (long long)bi * P.sA);
  const gptr32 B = (gptr32)(const void *)(reinterpret_cast<const float2 *>(P.B) + (long long)bi * P.sB);
  const int kbeg = ks * P.kchunk;
  const int kend = min(P.k, kbeg + P.kchunk);
  const int nkt = (kend > kbeg) ? (kend - kbeg + BK - 1) / BK : 0;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;

  // staging of one K tile (clamped loads, zero outside the problem)
  float2 fa[QA], fb[4];
  const auto load = [&](int k0) {
    if (OPA == OP_N) {  // A is m x k: column kk contiguous in i
      const int kk = tid >> 4, i = (tid & 15) * QA, kg = k0 + kk, kc = kg < kend ? kg : kend - 1;
#pragma unroll
      for (int q = 0; q < QA; ++q) {
        const int ig = m0 + i + q;
        const float2 v = ldg32(A + (long long)(ig < P.m ? ig : P.m - 1) + (long long)kc * P.lda);
        fa[q] = (ig < P.m && kg < kend) ? v : make_float2(0.f, 0.f);
      }
    } else {  // A is k x m (conjugate-transposed): row i contiguous in kk
      constexpr int TPR = NT / MB;
      const int i = tid / TPR, kk = (tid % TPR) * QA, ig = m0 + i, ic = ig < P.m ? ig : P.m - 1;
#pragma unroll
      for (int q = 0; q < QA; ++q) {
        const int kg = k0 + kk + q;
        const float2 v = ldg32(A + (long long)(kg < kend ? kg : kend - 1) + (long long)ic * P.lda);
        fa[q] = (ig < P.m && kg < kend) ? v : make_float2(0.f, 0.f);
      }
    }
    const int j = tid >> 2, kk = (tid & 3) * 4, jg = n0 + j, jc = jg < P.n ? jg : P.n - 1;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int kg = k0 + kk + q;
      const float2 v = ldg32(B + (long long)(kg < kend ? kg : kend - 1) + (long long)jc * P.ldb);
      fb[q] = (jg < P.n && kg < kend) ? v : make_float2(0.f, 0.f);
    }
  };
  const auto store = [&](int buf) {
    if (OPA == OP_N) {
      const int kk = tid >> 4, i = (tid & 15) * QA;
#pragma unroll
      for (int q = 0; q < QA; ++q) {
        As[buf][0][kk][i + q] = fa[q].x;
        As[buf][1][kk][i + q] = fa[q].y;
      }
    } else {
      constexpr int TPR = NT / MB;
      const int i = tid / TPR, kk = (tid % TPR) * QA;
#pragma unroll
      for (int q = 0; q < QA; ++q) {
        As[buf][0][kk + q][i] = fa[q].x;
        As[buf][1][kk + q][i] = -fa[q].y;  // conjugate
      }
    }
    const int j = tid >> 2, kk = (tid & 3) * 4;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      Bs[buf][0][kk + q][j] = fb[q].x;
      Bs[buf][1][kk + q][j] = fb[q].y;
    }
  };

  double sre[AW][2][4], sim[AW][2][4];
#pragma unroll
  for (int a = 0; a < AW; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) sre[a][b][r] = sim[a][b][r] = 0.0;
  if (nkt > 0) {
    load(kbeg);
    store(0);
  }
  __syncthreads();
  for (int kt = 0; kt < nkt; ++kt) {
    const int cur = kt & 1;
    load(kbeg + (kt + 1 < nkt ? kt + 1 : kt) * BK);
    __builtin_amdgcn_sched_barrier(0);
    f4 fre[AW][2], fim[AW][2];
#pragma unroll
    for (int a = 0; a < AW; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) fre[a][b] = fim[a][b] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kq = 0; kq < BK; kq += 4) {
      const int kk = kq + (lane >> 4);
      float ar[AW], ai[AW], nai[AW], br[2], bim[2];
#pragma unroll
      for (int a = 0; a < AW; ++a) {
        const int i = wm * (MB / 2) + a * 16 + (lane & 15);
        ar[a] = As[cur][0][kk][i];
        ai[a] = As[cur][1][kk][i];
        nai[a] = -ai[a];
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int j = wn * 32 + b * 16 + (lane & 15);
        br[b] = Bs[cur][0][kk][j];
        bim[b] = Bs[cur][1][kk][j];
      }
#pragma unroll
      for (int a = 0; a < AW; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          fre[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[a], br[b], fre[a][b], 0, 0, 0);
          fre[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(nai[a], bim[b], fre[a][b], 0, 0, 0);
          fim[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[a], bim[b], fim[a][b], 0, 0, 0);
          fim[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[a], br[b], fim[a][b], 0, 0, 0);
        }
    }
#pragma unroll
    for (int a = 0; a < AW; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          sre[a][b][r] += (double)fre[a][b][r];
          sim[a][b][r] += (double)fim[a][b][r];
        }
    if (kt + 1 < nkt) store(cur ^ 1);
    __syncthreads();
  }
  // output element of register r of v_mfma_f32_16x16x4f32: row 4 (lane / 16) + r, column lane % 16
  const auto row_of = [&](int a, int r) { return wm * (MB / 2) + a * 16 + 4 * (lane >> 4) + r; };
  const auto col_of = [&](int b) { return wn * 32 + b * 16 + (lane & 15); };
  if (P.ksplit == 1) {
    TO *C = reinterpret_cast<TO *>(P.C) + (long long)bi * P.sC;
    const bool rd = (P.beta.x != 0.0 || P.beta.y != 0.0);
#pragma unroll
    for (int a = 0; a < AW; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = m0 + row_of(a, r), j = n0 + col_of(b);
          if (i < P.m && j < P.n) {
            double2 v = cmul(P.alpha, make_double2(sre[a][b][r], sim[a][b][r]));
            TO *dst = C + (long long)i + (long long)j * P.ldc;
            if (rd) v = cfma(P.beta, to_d2(*dst), v);
            *dst = CT<TO>::from(v);
          }
        }
  } else if constexpr (sizeof(TO) == 16) {
    const long long tile_lin = ((long long)bi * P.tiles_n + tn) * P.tiles_m + tm;
    double2 *dst = partials + (P.part_off + tile_lin * P.ksplit + ks) * (long long)(BM * BN);
#pragma unroll
    for (int a = 0; a < AW; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) dst[col_of(b) * MB + row_of(a, r)] = make_double2(sre[a][b][r], sim[a][b][r]);
  }
}

template <bool TABLE>
hipError_t launch_impl(int opa, int opb, const ZBatch &b, const ZProb *table, const ZProb *host, int nprob,
                       int total_tiles, double2 *partials, int n_limit, hipStream_t s, int parts = 3,
                       bool fp32 = false, bool out32 = false) {
  if (total_tiles <= 0) return hipSuccess;
  const dim3 grid(total_tiles), block(NT);
  if (fp32 && (parts & 1)) {  // complex64 operands, op(B) = B, no column limit
    if (opb != OP_N || n_limit > 0) return hipErrorInvalidValue;
    if (out32)
      for (int i = 0; i < nprob; ++i)
        if (host[i].ksplit != 1) return hipErrorInvalidValue;  // complex64 C: unsplit problems only
#define LTD_CG(OA, TO)                                                                                        \
  do {                                                                                                        \
    if (host[0].bm == 32)                                                                                     \
      hipLaunchKernelGGL((cgemm32_kernel<OA, TABLE, 32, TO>), grid, block, 0, s, b, table, nprob, partials);   \
    else                                                                                                      \
      hipLaunchKernelGGL((cgemm32_kernel<OA, TABLE, 64, TO>), grid, block, 0, s, b, table, nprob, partials);   \
  } while (0)
    if (opa == OP_N && out32) LTD_CG(OP_N, float2);
    else if (opa == OP_N) LTD_CG(OP_N, double2);
    else if (out32) LTD_CG(OP_C, float2);
    else LTD_CG(OP_C, double2);
#undef LTD_CG
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    parts &= ~1;
  }
#define LTD_ZG(OA, OB)                                                                                         \
  do {                                                                                                         \
    if (host[0].bm == 32)                                                                                      \
      hipLaunchKernelGGL((zgemm_kernel<OA, OB, TABLE, 32>), grid, block, 0, s, b, table, nprob, partials, n_limit); \
    else                                                                                                       \
      hipLaunchKernelGGL((zgemm_kernel<OA, OB, TABLE, 64>), grid, block, 0, s, b, table, nprob, partials, n_limit); \
  } while (0)
  if (parts & 1) {
    if (opa == OP_N && opb == OP_N) LTD_ZG(OP_N, OP_N);
    else if (opa == OP_C && opb == OP_N) LTD_ZG(OP_C, OP_N);
    else if (opa == OP_N && opb == OP_C) LTD_ZG(OP_N, OP_C);
    else LTD_ZG(OP_C, OP_C);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
#undef LTD_ZG
  if (!(parts & 2)) return hipSuccess;
  bool split = false;
  int rtiles = 0;
  for (int i = 0; i < nprob; ++i) {
    split = split || host[i].ksplit > 1;
    rtiles = host[i].rtile_begin + host[i].tiles_m * host[i].tiles_n * host[i].batch;
  }
  if (!split) return hipSuccess;
  hipLaunchKernelGGL((zgemm_reduce<TABLE>), dim3(rtiles * ((BM * BN) / RED_T)), dim3(RED_T), 0, s, b, table, nprob,
                     partials, n_limit);
  return hipGetLastError();
}

}  // namespace

namespace {
// Plans the launch with output tiles of bm rows (see gemm_plan); returns the
// per-CU load estimate: blocks per CU x tile rows x K tiles per block.
long long plan_bm(ZProb *probs, int nprob, int bm, int target_blocks, long long max_part_tiles, int *total_tiles,
                  long long *part_tiles) {
  long long base_all = 0, base_split = 0;
  for (int i = 0; i < nprob; ++i) {
    ZProb &P = probs[i];
    P.bm = bm;
    P.tiles_m = (P.m + bm - 1) / bm;
    P.tiles_n = (P.n + BN - 1) / BN;
    if (P.batch < 1) P.batch = 1;
    base_all += (long long)P.tiles_m * P.tiles_n * P.batch;
  }
  const auto per_of = [](int kt) { return kt >= 64 ? 4 : (kt >= 16 ? 4 : 2); };
  int ks_common = 1;
  if (base_all > 0 && base_all < target_blocks) {
    for (int i = 0; i < nprob; ++i) {
      const ZProb &P = probs[i];
      const int kt = (P.k + BK - 1) / BK;
      if (kt >= 4) base_split += (long long)P.tiles_m * P.tiles_n * P.batch;
    }
    if (base_split > 0) {
      // rounded down: a launch of at most target_blocks leaves no tail round
      ks_common = (int)(target_blocks / base_all > 1 ? target_blocks / base_all : 1);
      const long long cap = max_part_tiles / base_split;
      if (ks_common > cap) ks_common = (int)(cap > 1 ? cap : 1);
    }
  }
  int tb = 0, rb = 0, kt_max = 0;
  long long part = 0;
  for (int i = 0; i < nprob; ++i) {
    ZProb &P = probs[i];
    const int base = P.tiles_m * P.tiles_n * P.batch;
    const int kt = (P.k + BK - 1) / BK;
    int ks = 1;
    if (ks_common > 1 && base > 0 && kt >= 4) {
      ks = ks_common < kt / per_of(kt) ? ks_common : kt / per_of(kt);
      if (ks < 1) ks = 1;
    }
    const int kt_per = (kt + ks - 1) / (ks > 0 ? ks : 1);
    P.kchunk = (kt_per > 0 ? kt_per : 1) * BK;
    P.ksplit = (P.k + P.kchunk - 1) / P.kchunk;
    if (P.ksplit < 1) P.ksplit = 1;
    P.tile_begin = tb;
    P.rtile_begin = rb;
    P.part_off = part;
    tb += base * P.ksplit;
    rb += base;
    if (P.ksplit > 1) part += (long long)base * P.ksplit;
    if (base > 0 && kt_per > kt_max) kt_max = kt_per;
  }
  // K-major order when every problem with tiles is split by the same factor
  int ks_all = 0;
  for (int i = 0; i < nprob && ks_all >= 0; ++i) {
    const ZProb &P = probs[i];
    if (P.tiles_m * P.tiles_n * P.batch == 0) continue;
    if (ks_all == 0) ks_all = P.ksplit;
    else if (P.ksplit != ks_all) ks_all = -1;
  }
  const int kmajor = (ks_all > 1 && (long long)rb * ks_all == tb) ? rb : 0;
  for (int i = 0; i < nprob; ++i) probs[i].kmajor = kmajor;
  *total_tiles = tb;
  *part_tiles = part;
  constexpr int CUS = 256;
  return (long long)((tb + CUS - 1) / CUS) * bm * (kt_max > 0 ? kt_max : 1);
}
}  // namespace

size_t gemm_plan(ZProb *probs, int nprob, int *total_tiles, int target_blocks, long long max_part_tiles) {
  // Output tiles of every problem; the K split is chosen for the launch as a
  // whole: the problems whose tiles alone leave the GPU short of target_blocks
  // split their K dimension by a common factor (at most K-tiles / per of each),
  // within the partial-tile budget.  The tile height (64 or 32 rows) is the one
  // with the lower per-CU load (ties: 64); 32-row tiles balance launches whose
  // 64-row tile count falls just past a multiple of the CU count, and waste less
  // on heights just past a multiple of 64.
  int t32 = 0, t64 = 0;
  long long p32 = 0, p64 = 0;
  const long long l32 = plan_bm(probs, nprob, 32, target_blocks, max_part_tiles, &t32, &p32);
  const long long l64 = plan_bm(probs, nprob, 64, target_blocks, max_part_tiles, &t64, &p64);
  long long part = p64;
  *total_tiles = t64;
  if (l32 < l64) {
    plan_bm(probs, nprob, 32, target_blocks, max_part_tiles, &t32, &p32);
    part = p32;
    *total_tiles = t32;
  }
  return (size_t)part * BM * BN * sizeof(double2);
}

hipError_t gemm_launch(int opa, int opb, const ZBatch &b, double2 *partials, hipStream_t s) {
  return launch_impl<false>(opa, opb, b, nullptr, b.p, b.nprob, b.total_tiles, partials, 0, s);
}

hipError_t gemm_launch_table(int opa, int opb, const ZProb *dev_table, const ZProb *host, int nprob,
                             int total_tiles, double2 *partials, int n_limit, hipStream_t s, int parts) {
  static const ZBatch empty{};
  return launch_impl<true>(opa, opb, empty, dev_table, host, nprob, total_tiles, partials, n_limit, s, parts);
}

hipError_t cgemm32_launch(int opa, const ZBatch &b, double2 *partials, hipStream_t s, bool out32) {
  return launch_impl<false>(opa, OP_N, b, nullptr, b.p, b.nprob, b.total_tiles, partials, 0, s, 3, true, out32);
}

hipError_t cgemm32_launch_table(int opa, const ZProb *dev_table, const ZProb *host, int nprob, int total_tiles,
                                double2 *partials, hipStream_t s, int parts, bool out32) {
  static const ZBatch empty{};
  return launch_impl<true>(opa, OP_N, empty, dev_table, host, nprob, total_tiles, partials, 0, s, parts, true,
                           out32);
}

}  // namespace ltd
