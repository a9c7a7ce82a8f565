// Interstitial part of the LAPW+LO operators by FFT convolution (Pela & Draxl,
// Sec. 2.3, second route; App. A, Eqs. (A.2), (A.4), (A.7)).
//
// For a block of plane-wave coefficient vectors the interstitial operators act
// as: transform to the real-space grid, multiply by the step function Theta
// (and by Theta V), transform back and read off at the G vectors:
//   S C  = F(Theta psi),  V C = F(Theta V psi),
//   T C  = 1/2 sum_i (G+k)_i F(Theta pi_i psi),  pi_i psi = F^{-1}((G+k)_i C),
//   Pz C = 1/2 [(G+k)_z F(Theta psi) + F(Theta pi_z psi)],
// with F f(q) = (1/N) sum_j f_j exp(-2 pi i q.j/N) and F^{-1} c = sum_q c_q
// exp(+2 pi i q.j/N).
//
// The coefficients live on a sphere that fills a few per cent of the grid, so
// each 3D transform is split into passes that only touch the box
// |g_i| <= b_i around it:
//   plane pass  (per kz in the box): 2D transform over (x, y); rows stream
//                through LDS in chunks, only the box columns stay in LDS
//                and only they are transformed along y;
//   line pass   (per tile of (x, y) positions): full-length z transforms in
//                LDS, fused with the pointwise products, so real-space fields
//                never reach HBM;
// and intermediate "slabs" hold nbz x N2 x N1 values per field and column.
//
// The 1D transforms are mixed-radix (8, 4, 5, 3, 2) Stockham autosort passes.
// Each wavefront owns whole lines, so a pass needs no block barrier: a
// wavefront reads all its butterfly inputs into registers, then writes the
// outputs (LDS operations of one wavefront complete in order).  The grid
// lengths of the workloads (16, 64, 72, 96, 160) are compile-time constants
// of their kernels, so all index arithmetic is strength-reduced; other lengths
// take a runtime-length path.
#include "common.h"

#include <cmath>
#include <numeric>
#include <type_traits>

namespace ltd {

namespace {

constexpr int FFT_NT = 256;
constexpr double SQ1_2 = 0.70710678118654752440;  // 1/sqrt(2)
constexpr double SQ3_2 = 0.86602540378443864676;  // sqrt(3)/2
constexpr double C5_1 = 0.30901699437494742410;   // cos(2 pi/5)
constexpr double C5_2 = -0.80901699437494742410;  // cos(4 pi/5)
constexpr double S5_1 = 0.95105651629515357212;   // sin(2 pi/5)
constexpr double S5_2 = 0.58778525229247312917;   // sin(4 pi/5)

template <int DIR, class T>
__device__ inline T mul_i(T a) {  // (DIR i) * a
  return DIR > 0 ? CT<T>::mk(-a.y, a.x) : CT<T>::mk(a.y, -a.x);
}

template <int DIR, class T>
__device__ inline void dft4(T &v0, T &v1, T &v2, T &v3) {
  const T a = cadd(v0, v2), b = csub(v0, v2), c = cadd(v1, v3), d = mul_i<DIR>(csub(v1, v3));
  v0 = cadd(a, c);
  v2 = csub(a, c);
  v1 = cadd(b, d);
  v3 = csub(b, d);
}

template <int DIR, class T>
__device__ inline void dft8(T *v) {
  using R = typename CT<T>::R;
  const R h = (R)SQ1_2;
  T e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  T o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4<DIR>(e0, e1, e2, e3);
  dft4<DIR>(o0, o1, o2, o3);
  // twiddles w8^p, w8 = exp(DIR i pi/4)
  const T t1 = CT<T>::mk(h * (o1.x - DIR * o1.y), h * (o1.y + DIR * o1.x));
  const T t2 = mul_i<DIR>(o2);
  const T t3 = CT<T>::mk(h * (-o3.x - DIR * o3.y), h * (-o3.y + DIR * o3.x));
  v[0] = cadd(e0, o0);
  v[4] = csub(e0, o0);
  v[1] = cadd(e1, t1);
  v[5] = csub(e1, t1);
  v[2] = cadd(e2, t2);
  v[6] = csub(e2, t2);
  v[3] = cadd(e3, t3);
  v[7] = csub(e3, t3);
}

// Length-8 DFT whose inputs 2..5 are zero (only v[0], v[1], v[6], v[7] read).
template <int DIR, class T>
__device__ __forceinline__ void dft8_z2345(T *v) {
  using R = typename CT<T>::R;
  const R h = (R)SQ1_2;
  // the two length-4 DFTs of (v0, 0, 0, v6) and (v1, 0, 0, v7)
  const T e0 = cadd(v[0], v[6]), e2 = csub(v[0], v[6]);
  const T e1 = csub(v[0], mul_i<DIR>(v[6])), e3 = cadd(v[0], mul_i<DIR>(v[6]));
  const T o0 = cadd(v[1], v[7]), o2 = csub(v[1], v[7]);
  const T o1 = csub(v[1], mul_i<DIR>(v[7])), o3 = cadd(v[1], mul_i<DIR>(v[7]));
  const T t1 = CT<T>::mk(h * (o1.x - DIR * o1.y), h * (o1.y + DIR * o1.x));
  const T t2 = mul_i<DIR>(o2);
  const T t3 = CT<T>::mk(h * (-o3.x - DIR * o3.y), h * (-o3.y + DIR * o3.x));
  v[0] = cadd(e0, o0);
  v[4] = csub(e0, o0);
  v[1] = cadd(e1, t1);
  v[5] = csub(e1, t1);
  v[2] = cadd(e2, t2);
  v[6] = csub(e2, t2);
  v[3] = cadd(e3, t3);
  v[7] = csub(e3, t3);
}

template <int DIR, class T>
__device__ inline void dft3(T *v) {
  using R = typename CT<T>::R;
  const T t = cadd(v[1], v[2]);
  const T m = CT<T>::mk(v[0].x - (R)0.5 * t.x, v[0].y - (R)0.5 * t.y);
  const T u = cscale(mul_i<DIR>(csub(v[1], v[2])), (R)SQ3_2);
  v[0] = cadd(v[0], t);
  v[1] = cadd(m, u);
  v[2] = csub(m, u);
}

template <int DIR, class T>
__device__ inline void dft5(T *v) {
  using R = typename CT<T>::R;
  const R c1 = (R)C5_1, c2 = (R)C5_2, s1 = (R)S5_1, s2 = (R)S5_2;
  const T a1 = cadd(v[1], v[4]), a2 = cadd(v[2], v[3]);
  const T b1 = csub(v[1], v[4]), b2 = csub(v[2], v[3]);
  const T y0 = cadd(v[0], cadd(a1, a2));
  const T m1 = CT<T>::mk(v[0].x + c1 * a1.x + c2 * a2.x, v[0].y + c1 * a1.y + c2 * a2.y);
  const T m2 = CT<T>::mk(v[0].x + c2 * a1.x + c1 * a2.x, v[0].y + c2 * a1.y + c1 * a2.y);
  const T n1 = mul_i<DIR>(CT<T>::mk(s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y));
  const T n2 = mul_i<DIR>(CT<T>::mk(s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y));
  v[0] = y0;
  v[1] = cadd(m1, n1);
  v[4] = csub(m1, n1);
  v[2] = cadd(m2, n2);
  v[3] = csub(m2, n2);
}

// In-place DFT of length R: y_p = sum_q v_q exp(DIR 2 pi i p q / R).
template <int R, int DIR, class T>
__device__ inline void dft_small(T *v) {
  if constexpr (R == 2) {
    const T a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 3) {
    dft3<DIR>(v);
  } else if constexpr (R == 4) {
    dft4<DIR>(v[0], v[1], v[2], v[3]);
  } else if constexpr (R == 5) {
    dft5<DIR>(v);
  } else {
    static_assert(R == 8, "radix");
    dft8<DIR>(v);
  }
}

constexpr double C9_1 = 0.76604444311897803520;   // cos(2 pi/9)
constexpr double S9_1 = 0.64278760968653932632;   // sin(2 pi/9)
constexpr double C9_2 = 0.17364817766693034885;   // cos(4 pi/9)
constexpr double S9_2 = 0.98480775301220805937;   // sin(4 pi/9)
constexpr double C9_4 = -0.93969262078590838405;  // cos(8 pi/9)
constexpr double S9_4 = 0.34202014332566873304;   // sin(8 pi/9)

// Length 9 as 3 x 3: input q = 3 q1 + q2, output p = p1 + 3 p2.
template <int DIR, class T>
__device__ inline void dft9(T *v) {
  using R = typename CT<T>::R;
  T a[3][3];
#pragma unroll
  for (int q2 = 0; q2 < 3; ++q2) {
    T t[3] = {v[q2], v[3 + q2], v[6 + q2]};
    dft3<DIR>(t);
    a[q2][0] = t[0];
    a[q2][1] = t[1];
    a[q2][2] = t[2];
  }
  a[1][1] = cmul(a[1][1], CT<T>::mk((R)C9_1, (R)(DIR * S9_1)));
  a[1][2] = cmul(a[1][2], CT<T>::mk((R)C9_2, (R)(DIR * S9_2)));
  a[2][1] = cmul(a[2][1], CT<T>::mk((R)C9_2, (R)(DIR * S9_2)));
  a[2][2] = cmul(a[2][2], CT<T>::mk((R)C9_4, (R)(DIR * S9_4)));
#pragma unroll
  for (int p1 = 0; p1 < 3; ++p1) {
    T t[3] = {a[0][p1], a[1][p1], a[2][p1]};
    dft3<DIR>(t);
    v[p1] = t[0];
    v[p1 + 3] = t[1];
    v[p1 + 6] = t[2];
  }
}

// Length 12 as 3 x 4: input q = 4 q1 + q2, output p = p1 + 3 p2:
//   y[p1 + 3 p2] = sum_q2 w4^(p2 q2) w12^(p1 q2) sum_q1 w3^(p1 q1) v[4 q1 + q2].
template <int DIR, class T>
__device__ inline void dft12(T *v) {
  using R = typename CT<T>::R;
  T a[4][3];
#pragma unroll
  for (int q2 = 0; q2 < 4; ++q2) {
    T t[3] = {v[q2], v[4 + q2], v[8 + q2]};
    dft3<DIR>(t);
    a[q2][0] = t[0];
    a[q2][1] = t[1];
    a[q2][2] = t[2];
  }
  // w12^e, e = p1 q2: 1 = (sqrt3/2, 1/2), 2 = (1/2, sqrt3/2), 3 = i, 4 = (-1/2, sqrt3/2), 6 = -1
  // (imaginary parts times DIR)
  a[1][1] = cmul(a[1][1], CT<T>::mk((R)SQ3_2, (R)(DIR * 0.5)));
  a[2][1] = cmul(a[2][1], CT<T>::mk((R)0.5, (R)(DIR * SQ3_2)));
  a[3][1] = mul_i<DIR>(a[3][1]);
  a[1][2] = cmul(a[1][2], CT<T>::mk((R)0.5, (R)(DIR * SQ3_2)));
  a[2][2] = cmul(a[2][2], CT<T>::mk((R)-0.5, (R)(DIR * SQ3_2)));
  a[3][2] = CT<T>::mk(-a[3][2].x, -a[3][2].y);
#pragma unroll
  for (int p1 = 0; p1 < 3; ++p1) {
    T t0 = a[0][p1], t1 = a[1][p1], t2 = a[2][p1], t3 = a[3][p1];
    dft4<DIR>(t0, t1, t2, t3);
    v[p1] = t0;
    v[p1 + 3] = t1;
    v[p1 + 6] = t2;
    v[p1 + 9] = t3;
  }
}

// Length-12 DFT whose inputs 3..8 are zero (only v[0..2], v[9..11] read), the
// first pass of a 108 = 12 x 9 line when the box half-width is at most 26: in the
// 3 x 4 form the length-3 columns (v[q2], v[4+q2], v[8+q2]) have known zeros.
template <int DIR, class T>
__device__ inline void dft12_z3to8(T *v) {
  using R = typename CT<T>::R;
  T a[4][3];
  a[0][0] = a[0][1] = a[0][2] = v[0];  // (v0, 0, 0)
#pragma unroll
  for (int q2 = 1; q2 <= 2; ++q2) {  // (v[q2], 0, v[8+q2])
    const T x = v[q2], z = v[8 + q2];
    const T m = CT<T>::mk(x.x - (R)0.5 * z.x, x.y - (R)0.5 * z.y);
    const T u = cscale(mul_i<DIR>(CT<T>::mk(-z.x, -z.y)), (R)SQ3_2);
    a[q2][0] = cadd(x, z);
    a[q2][1] = cadd(m, u);
    a[q2][2] = csub(m, u);
  }
  {  // (0, 0, v11)
    const T z = v[11];
    const T m = CT<T>::mk((R)-0.5 * z.x, (R)-0.5 * z.y);
    const T u = cscale(mul_i<DIR>(CT<T>::mk(-z.x, -z.y)), (R)SQ3_2);
    a[3][0] = z;
    a[3][1] = cadd(m, u);
    a[3][2] = csub(m, u);
  }
  a[1][1] = cmul(a[1][1], CT<T>::mk((R)SQ3_2, (R)(DIR * 0.5)));
  a[2][1] = cmul(a[2][1], CT<T>::mk((R)0.5, (R)(DIR * SQ3_2)));
  a[3][1] = mul_i<DIR>(a[3][1]);
  a[1][2] = cmul(a[1][2], CT<T>::mk((R)0.5, (R)(DIR * SQ3_2)));
  a[2][2] = cmul(a[2][2], CT<T>::mk((R)-0.5, (R)(DIR * SQ3_2)));
  a[3][2] = CT<T>::mk(-a[3][2].x, -a[3][2].y);
#pragma unroll
  for (int p1 = 0; p1 < 3; ++p1) {
    T t0 = a[0][p1], t1 = a[1][p1], t2 = a[2][p1], t3 = a[3][p1];
    dft4<DIR>(t0, t1, t2, t3);
    v[p1] = t0;
    v[p1 + 3] = t1;
    v[p1 + 6] = t2;
    v[p1 + 9] = t3;
  }
}

// In-register DFT of the lengths the two-factor transforms use.
template <int R, int DIR, class T>
__device__ __forceinline__ void dft_reg(T *v) {
  if constexpr (R == 9) dft9<DIR>(v);
  else if constexpr (R == 12) dft12<DIR>(v);
  else if constexpr (R == 1) (void)v;
  else dft_small<R, DIR>(v);
}

template <int R>
struct Tpl {  // butterflies per lane and stage (register budget)
  static constexpr int value = (R == 8) ? 1 : (R == 5) ? 1 : (R == 4) ? 2 : (R == 3) ? 2 : 4;
};

__host__ __device__ constexpr int tpl_of(int r) { return r == 8 ? 1 : r == 5 ? 1 : r == 4 ? 2 : r == 3 ? 2 : 4; }

struct Radices {
  int n;
  int r[FFT_MAXST];
};

__host__ __device__ constexpr Radices factor_len(int L) {
  Radices f{0, {0, 0, 0, 0, 0, 0, 0, 0}};
  const int order[5] = {8, 4, 5, 3, 2};
  int x = L;
  for (int oi = 0; oi < 5; ++oi)
    while (x > 1 && x % order[oi] == 0 && f.n < FFT_MAXST) {
      f.r[f.n++] = order[oi];
      x /= order[oi];
    }
  return f;
}

// Largest number of lines one wavefront can transform per pass.
__host__ __device__ constexpr int lpw_len(int L) {
  const Radices f = factor_len(L);
  int best = 1 << 20;
  for (int s = 0; s < f.n; ++s) {
    const int v = (64 * tpl_of(f.r[s])) / (L / f.r[s]);
    best = v < best ? v : best;
  }
  return best < 1 ? 1 : best;
}

__host__ __device__ inline int lines_per_wave(const FftPlan &p) {
  int best = 1 << 20;
  for (int s = 0; s < p.nst; ++s) {
    const int r = p.radix[s];
    const int v = (64 * tpl_of(r)) / (p.L / r);
    best = v < best ? v : best;
  }
  return best < 1 ? 1 : best;
}

// Line addressing: element e of line l sits at buf[map(l) + e * es].
struct LinesUniform {
  int base, ls;
  __device__ int operator()(int l) const { return base + l * ls; }
};
struct LinesTwo {  // lines [0, h) at a0 + l, lines [h, 2h) at a1 + (l - h)
  int a0, a1, h;
  __device__ int operator()(int l) const { return l < h ? a0 + l : a1 + (l - h); }
};

// One Stockham pass of radix R on the lines [l0, l0 + nl) of this wavefront.
// L, NS: compile-time line length and sub-transform size when L > 0.
template <int R, int DIR, int L, int NS, class LM, class T>
__device__ __forceinline__ void fft_stage(T *buf, const LM &lm, int l0, int nl, int es, int Lr, int NSr,
                                 const T *tw, int lane) {
  constexpr int TPL = Tpl<R>::value;
  const int len = (L > 0) ? L : Lr;
  const int ns = (L > 0) ? NS : NSr;
  const int nb = len / R;
  const int ntask = nl * nb;
  const int twm = len / (ns * R);
  T v[TPL][R];
  int ob[TPL];
#pragma unroll
  for (int t = 0; t < TPL; ++t) {
    const int task = lane + 64 * t;
    ob[t] = -1;
    if (task < ntask) {
      const int line = task / nb;
      const int j = task - line * nb;
      const int k = j % ns;
      const int base = lm(l0 + line);
      const int tws = twm * k;  // tws * q < len for q < R
#pragma unroll
      for (int q = 0; q < R; ++q) {
        T x = buf[base + (j + q * nb) * es];
        if (q > 0) {
          T w = tw[tws * q];
          if (DIR > 0) w.y = -w.y;
          x = cmul(x, w);
        }
        v[t][q] = x;
      }
      ob[t] = base + ((j / ns) * ns * R + k) * es;
    }
  }
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
#pragma unroll
  for (int t = 0; t < TPL; ++t) {
    if (ob[t] >= 0) {
      dft_small<R, DIR>(v[t]);
#pragma unroll
      for (int q = 0; q < R; ++q) buf[ob[t] + q * ns * es] = v[t][q];
    }
  }
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

template <int DIR, int L, int S, int NS, class LM, class T>
__device__ __forceinline__ void fft_stages_ct(T *buf, const LM &lm, int l0, int nl, int es, const T *tw,
                                     int lane) {
  constexpr Radices f = factor_len(L);
  if constexpr (S < f.n) {
    constexpr int R = f.r[S];
    fft_stage<R, DIR, L, NS>(buf, lm, l0, nl, es, L, NS, tw, lane);
    fft_stages_ct<DIR, L, S + 1, NS * R>(buf, lm, l0, nl, es, tw, lane);
  }
}

template <int DIR, class LM, class T>
__device__ __forceinline__ void fft_stages_rt(T *buf, const LM &lm, int l0, int nl, int es, const FftPlan &p,
                              const T *tw, int lane) {
  int ns = 1;
  for (int s = 0; s < p.nst; ++s) {
    const int r = p.radix[s];
    switch (r) {
      case 8: fft_stage<8, DIR, 0, 0>(buf, lm, l0, nl, es, p.L, ns, tw, lane); break;
      case 4: fft_stage<4, DIR, 0, 0>(buf, lm, l0, nl, es, p.L, ns, tw, lane); break;
      case 5: fft_stage<5, DIR, 0, 0>(buf, lm, l0, nl, es, p.L, ns, tw, lane); break;
      case 3: fft_stage<3, DIR, 0, 0>(buf, lm, l0, nl, es, p.L, ns, tw, lane); break;
      default: fft_stage<2, DIR, 0, 0>(buf, lm, l0, nl, es, p.L, ns, tw, lane); break;
    }
    ns *= r;
  }
}

// All waves of the block transform `nlines` lines (length L, or p.L when L == 0);
// ends with a block barrier.
template <int DIR, int L, class LM, class T>
__device__ __forceinline__ void fft_block(T *buf, const LM &lm, int nlines, int es, const FftPlan &p, const T *tw) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if constexpr (L > 0) {
    constexpr int lpw = lpw_len(L);
    for (int l0 = wave * lpw; l0 < nlines; l0 += nw * lpw) {
      const int nl = (nlines - l0) < lpw ? (nlines - l0) : lpw;
      fft_stages_ct<DIR, L, 0, 1>(buf, lm, l0, nl, es, tw, lane);
    }
  } else {
    const int lpw = lines_per_wave(p);
    for (int l0 = wave * lpw; l0 < nlines; l0 += nw * lpw) {
      const int nl = (nlines - l0) < lpw ? (nlines - l0) : lpw;
      fft_stages_rt<DIR>(buf, lm, l0, nl, es, p, tw, lane);
    }
  }
  __syncthreads();
}

template <class T>
__device__ inline void load_tw(T *dst, const double2 *src, int L) {
  for (int i = threadIdx.x; i < L; i += blockDim.x) dst[i] = CT<T>::from(src[i]);
}

// box index of a kx column (x = kx mod n1): kx + bx, or -1 outside the box
__device__ inline int box_of(int x, int n1, int bx) {
  return x <= bx ? x + bx : (x >= n1 - bx ? x - n1 + bx : -1);
}

// ---------------------------------------------------------------------------
// Inverse plane pass: sphere coefficients (times 1 or (G+k)_i) -> slab planes.
// grid (nbz, ncols, nk); fields: 0 psi, 1..3 pi_x, pi_y, pi_z.
// LDS: box columns bx_[nbx][n2+1], a chunk of rows rw[ch][n1+1], twiddles.
// ---------------------------------------------------------------------------
template <int L1, int L2>
__global__ __launch_bounds__(FFT_NT) void k_inv_plane(const Grid g, const FftKArgs ka, int ncols, int nfields,
                                                      int ch) {
  extern __shared__ double2 sm[];
  const int pz = blockIdx.x, col = blockIdx.y, kk = blockIdx.z;
  const int n1 = L1 > 0 ? L1 : g.n1, n2 = L2 > 0 ? L2 : g.n2;
  const int bx = g.bx, nbx = g.nbx;
  const int bp = n2 + 1, rp = n1 + 1;
  double2 *bxc = sm;
  double2 *rw = bxc + nbx * bp;
  double2 *tw1 = rw + ch * rp;
  double2 *tw2 = tw1 + n1;
  load_tw(tw1, g.tw1, n1);
  load_tw(tw2, g.tw2, n2);
  const KSphere &sp = ka.sph[kk];
  const InvIn in = ka.in[kk];
  const int p0 = sp.plane_ptr[pz], p1 = sp.plane_ptr[pz + 1];
  const long long plane_sz = (long long)n1 * n2;
  const long long fstride = (long long)ncols * g.nbz * plane_sz;
  double2 *out = ka.slab_out[kk] + ((long long)col * g.nbz + pz) * plane_sz;
  for (int f = 0; f < nfields; ++f) {
    for (int i = threadIdx.x; i < nbx * bp; i += blockDim.x) bxc[i] = make_double2(0.0, 0.0);
    __syncthreads();
    for (int i = p0 + threadIdx.x; i < p1; i += blockDim.x) {
      const int gi = sp.pts_g[i], xy = sp.pts_xy[i];
      double2 c = in.c[(long long)gi + (long long)col * in.ldc];
      if (f > 0) c = cscale(c, sp.gk[3 * gi + (f - 1)]);
      const int y = xy / n1, x = xy - y * n1;
      bxc[box_of(x, n1, bx) * bp + y] = c;
    }
    __syncthreads();
    fft_block<1, L2>(bxc, LinesUniform{0, bp}, nbx, 1, g.p2, tw2);  // along y, box columns
    double2 *o = out + f * fstride;
    for (int y0 = 0; y0 < n2; y0 += ch) {
      const int nr = (n2 - y0) < ch ? (n2 - y0) : ch;
      for (int i = threadIdx.x; i < nr * n1; i += blockDim.x) {
        const int r = i / n1, x = i - r * n1;
        const int b = box_of(x, n1, bx);
        rw[r * rp + x] = (b >= 0) ? bxc[b * bp + y0 + r] : make_double2(0.0, 0.0);
      }
      __syncthreads();
      fft_block<1, L1>(rw, LinesUniform{0, rp}, nr, 1, g.p1, tw1);  // along x
      for (int i = threadIdx.x; i < nr * n1; i += blockDim.x) {
        const int r = i / n1, x = i - r * n1;
        o[(long long)(y0 + r) * n1 + x] = rw[r * rp + x];
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// Line pass along z for a tile of T consecutive (x, y) positions.
// MODE_V:    in field 0 (psi)                 -> out field 0 (Theta V psi)
// otherwise: in fields psi, pi_x, pi_y, pi_z -> out Theta psi, Theta V psi,
//            Theta pi_x psi, Theta pi_y psi, Theta pi_z psi
// LDS: A [n3][T+1] (and B [n3][T+1] unless MODE_V), twiddles.
// ---------------------------------------------------------------------------
template <int L3, bool VMODE>
__global__ __launch_bounds__(FFT_NT) void k_lines(const Grid g, const FftKArgs ka, int ncols, int T,
                                                  const double *__restrict__ thv) {
  extern __shared__ double2 sm[];
  const int tile = blockIdx.x, col = blockIdx.y, kk = blockIdx.z;
  const int n3 = L3 > 0 ? L3 : g.n3;
  const int nbz = g.nbz, bz = g.bz;
  const long long plane_sz = (long long)g.n1 * g.n2;
  const int pos0 = tile * T;
  const int tp = T + 1;
  constexpr bool vmode = VMODE;
  double2 *A = sm;
  double2 *B = sm + n3 * tp;
  double2 *tw3 = vmode ? B : B + n3 * tp;
  load_tw(tw3, g.tw3, n3);
  const long long fstride = (long long)ncols * nbz * plane_sz;
  const double2 *in = ka.slab_in[kk] + (long long)col * nbz * plane_sz;
  double2 *out = ka.slab_out[kk] + (long long)col * nbz * plane_sz;
  const int ntot = nbz * T;

  // zero-fills the line buffer and places the box of kz values at z = kz mod n3
  auto load_field = [&](const double2 *src) {
    for (int i = threadIdx.x; i < n3 * T; i += blockDim.x) {
      const int z = i / T, t = i - z * T;
      const int kz = z <= bz ? z : z - n3;
      double2 v = make_double2(0.0, 0.0);
      if ((kz >= -bz && kz <= bz) && pos0 + t < plane_sz) v = src[(long long)(kz + bz) * plane_sz + pos0 + t];
      A[z * tp + t] = v;
    }
    __syncthreads();
  };
  auto store_field = [&](const double2 *buf, double2 *dst) {
    for (int i = threadIdx.x; i < ntot; i += blockDim.x) {
      const int p = i / T, t = i - p * T;
      const int kz = p - bz;
      const int z = kz < 0 ? kz + n3 : kz;
      if (pos0 + t < plane_sz) dst[(long long)p * plane_sz + pos0 + t] = buf[z * tp + t];
    }
  };

  if constexpr (VMODE) {
    load_field(in);
    fft_block<1, L3>(A, LinesUniform{0, 1}, T, tp, g.p3, tw3);
    for (int i = threadIdx.x; i < n3 * T; i += blockDim.x) {
      const int z = i / T, t = i - z * T;
      if (pos0 + t < plane_sz) A[z * tp + t] = cscale(A[z * tp + t], thv[(long long)z * plane_sz + pos0 + t]);
    }
    __syncthreads();
    fft_block<-1, L3>(A, LinesUniform{0, 1}, T, tp, g.p3, tw3);
    store_field(A, out);
    return;
  } else {
  // psi -> Theta psi, Theta V psi
  load_field(in);
  fft_block<1, L3>(A, LinesUniform{0, 1}, T, tp, g.p3, tw3);
  for (int i = threadIdx.x; i < n3 * T; i += blockDim.x) {
    const int z = i / T, t = i - z * T;
    double th = 0.0, tv = 0.0;
    if (pos0 + t < plane_sz) {
      const long long gidx = (long long)z * plane_sz + pos0 + t;
      th = g.theta[gidx];
      tv = thv[gidx];
    }
    const double2 a = A[z * tp + t];
    B[z * tp + t] = cscale(a, tv);
    A[z * tp + t] = cscale(a, th);
  }
  __syncthreads();
  fft_block<-1, L3>(A, LinesTwo{0, n3 * tp, T}, 2 * T, tp, g.p3, tw3);
  store_field(A, out);
  store_field(B, out + fstride);
  __syncthreads();
  for (int f = 1; f <= 3; ++f) {
    load_field(in + f * fstride);
    fft_block<1, L3>(A, LinesUniform{0, 1}, T, tp, g.p3, tw3);
    for (int i = threadIdx.x; i < n3 * T; i += blockDim.x) {
      const int z = i / T, t = i - z * T;
      const double th = (pos0 + t < plane_sz) ? g.theta[(long long)z * plane_sz + pos0 + t] : 0.0;
      A[z * tp + t] = cscale(A[z * tp + t], th);
    }
    __syncthreads();
    fft_block<-1, L3>(A, LinesUniform{0, 1}, T, tp, g.p3, tw3);
    store_field(A, out + (f + 1) * fstride);
    __syncthreads();
  }
  }
}

// ---------------------------------------------------------------------------
// Forward plane pass: slab planes -> values at the sphere, combined per mode.
// ---------------------------------------------------------------------------
// The value of output field f at sphere point gi of column col into the mode's
// outputs: MODE_V Y; MODE_HS S C and H C = F(Th V psi) + (A/c) F(1/2 (gz Th psi
// + Th pi_z psi)) + (A^2 / 2 c^2) F(Th psi) + sum_i 1/2 (G+k)_i F(Th pi_i psi);
// MODE_TVPS the blocks T, V, P, S applied separately.
__device__ __forceinline__ void fwd_out_point(const FwdOut &fo, const KSphere &sp, int gi, int col, int f, int mode,
                                              double2 val, double alpha_a, double beta_a) {
  const long long c = (long long)col;
  if (mode == FFT_MODE_V) {
    fo.o0[gi + c * fo.ld0] = val;
  } else if (mode == FFT_MODE_HS) {
    double2 *hc = fo.o0 + gi + c * fo.ld0;
    const double gz = sp.gk[3 * gi + 2];
    if (f == 0) {
      fo.o1[gi + c * fo.ld1] = val;                    // S C
      *hc = cscale(val, alpha_a * 0.5 * gz + beta_a);  // (A/c) 1/2 gz F(Th psi) + (A^2/2c^2) F(Th psi)
    } else if (f == 1) {
      *hc = cadd(*hc, val);                            // F(Th V psi)
    } else {
      double w = 0.5 * sp.gk[3 * gi + (f - 2)];        // 1/2 (G+k)_i F(Th pi_i psi)
      if (f == 4) w += 0.5 * alpha_a;                  // (A/c) 1/2 F(Th pi_z psi)
      *hc = cadd(*hc, cscale(val, w));
    }
  } else {  // TVPS
    const double gz = sp.gk[3 * gi + 2];
    if (f == 0) {
      fo.o3[gi + c * fo.ld3] = val;                    // S
      fo.o2[gi + c * fo.ld2] = cscale(val, 0.5 * gz);  // P part
    } else if (f == 1) {
      fo.o1[gi + c * fo.ld1] = val;                    // V
    } else {
      const double w = 0.5 * sp.gk[3 * gi + (f - 2)];
      double2 *t = fo.o0 + gi + c * fo.ld0;
      *t = (f == 2) ? cscale(val, w) : cadd(*t, cscale(val, w));
      if (f == 4) {
        double2 *p = fo.o2 + gi + c * fo.ld2;
        *p = cadd(*p, cscale(val, 0.5));
      }
    }
  }
}
template <int L1, int L2>
__global__ __launch_bounds__(FFT_NT) void k_fwd_plane(const Grid g, const FftKArgs ka, int ncols, int mode,
                                                      double alpha_a, double beta_a, int ch) {
  extern __shared__ double2 sm[];
  const int pz = blockIdx.x, col = blockIdx.y, kk = blockIdx.z;
  const int n1 = L1 > 0 ? L1 : g.n1, n2 = L2 > 0 ? L2 : g.n2;
  const int bx = g.bx, nbx = g.nbx;
  const int bp = n2 + 1, rp = n1 + 1;
  double2 *bxc = sm;
  double2 *rw = bxc + nbx * bp;
  double2 *tw1 = rw + ch * rp;
  double2 *tw2 = tw1 + n1;
  load_tw(tw1, g.tw1, n1);
  load_tw(tw2, g.tw2, n2);
  const KSphere &sp = ka.sph[kk];
  const FwdOut &fo = ka.out[kk];
  const int p0 = sp.plane_ptr[pz], p1 = sp.plane_ptr[pz + 1];
  const long long plane_sz = (long long)n1 * n2;
  const long long fstride = (long long)ncols * g.nbz * plane_sz;
  const double2 *src0 = ka.slab_in[kk] + ((long long)col * g.nbz + pz) * plane_sz;
  const double inv_n = 1.0 / ((double)n1 * n2 * g.n3);
  const int nf = (mode == FFT_MODE_V) ? 1 : 5;
  __syncthreads();
  for (int f = 0; f < nf; ++f) {
    const double2 *src = src0 + f * fstride;
    for (int y0 = 0; y0 < n2; y0 += ch) {
      const int nr = (n2 - y0) < ch ? (n2 - y0) : ch;
      for (int i = threadIdx.x; i < nr * n1; i += blockDim.x) {
        const int r = i / n1, x = i - r * n1;
        rw[r * rp + x] = src[(long long)(y0 + r) * n1 + x];
      }
      __syncthreads();
      fft_block<-1, L1>(rw, LinesUniform{0, rp}, nr, 1, g.p1, tw1);  // along x
      for (int i = threadIdx.x; i < nr * nbx; i += blockDim.x) {
        const int r = i / nbx, b = i - r * nbx;
        const int kx = b - bx;
        bxc[b * bp + y0 + r] = rw[r * rp + (kx < 0 ? kx + n1 : kx)];
      }
      __syncthreads();
    }
    fft_block<-1, L2>(bxc, LinesUniform{0, bp}, nbx, 1, g.p2, tw2);  // along y, box columns
    for (int i = p0 + threadIdx.x; i < p1; i += blockDim.x) {
      const int gi = sp.pts_g[i], xy = sp.pts_xy[i];
      const int y = xy / n1, x = xy - y * n1;
      fwd_out_point(fo, sp, gi, col, f, mode, cscale(bxc[box_of(x, n1, bx) * bp + y], inv_n), alpha_a, beta_a);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Per-step rebuild path.  The cached grid image of the auxiliary basis is kept
// transformed along y only: per column the box array c[kz][y][kx] (kz, kx in the
// G box, y over the grid).  A step then runs
//   k_rb_xz (per y plane): inverse x transforms of the nbz rows, inverse z
//     transforms of the x columns, product with Theta V, forward z and x
//     transforms, box read-out -> d[kz][y][kx];
//   k_rb_y (per kz plane): forward y transforms of the box columns and the
//     sphere read-out, row i of Y holding sphere-table point i (plane order,
//     contiguous writes; the projection takes Phi~'s G rows in that order),
// so a column moves 3 box arrays (nbz*N2*nbx values) through HBM per step.
// ---------------------------------------------------------------------------

// Setup: sphere coefficients of one kz plane -> inverse y transforms of the box
// columns -> c[kz][y][kx].  grid (nbz, ncols, nk).
// T: element type of the cache (double2, or float2 for the FP32 residual).
template <int L2, class T>
__global__ __launch_bounds__(FFT_NT) void k_rb_cache(const Grid g, const FftKArgs ka, int ncols) {
  extern __shared__ double2 sm_raw[];
  T *sm = reinterpret_cast<T *>(sm_raw);
  const int pz = blockIdx.x, col = blockIdx.y, kk = blockIdx.z;
  const int n2 = L2 > 0 ? L2 : g.n2;
  const int bx = g.bx, nbx = g.nbx;
  const int bp = n2 + 1;
  T *bxc = sm;
  T *tw2 = bxc + nbx * bp;
  load_tw(tw2, g.tw2, n2);
  const KSphere &sp = ka.sph[kk];
  const InvIn in = ka.in[kk];
  const int p0 = sp.plane_ptr[pz], p1 = sp.plane_ptr[pz + 1];
  for (int i = threadIdx.x; i < nbx * bp; i += blockDim.x) bxc[i] = CT<T>::mk(0, 0);
  __syncthreads();
  for (int i = p0 + threadIdx.x; i < p1; i += blockDim.x) {
    const int gi = sp.pts_g[i], xy = sp.pts_xy[i];
    const int y = xy / g.d1, x = xy - y * g.d1;
    const int yr = y <= g.by ? y : y - g.d2 + n2;  // k_y mod n2
    bxc[box_of(x, g.d1, bx) * bp + yr] = CT<T>::from(in.c[(long long)gi + (long long)col * in.ldc]);
  }
  __syncthreads();
  fft_block<1, L2>(bxc, LinesUniform{0, bp}, nbx, 1, g.p2, tw2);
  const long long csz = (long long)g.nbz * n2 * nbx;
  T *out = reinterpret_cast<T *>(ka.slab_out[kk]) + (long long)col * csz + (long long)pz * n2 * nbx;
  for (int i = threadIdx.x; i < n2 * nbx; i += blockDim.x) {
    const int y = i / nbx, b = i - y * nbx;
    out[i] = bxc[b * bp + y];
  }
}

// Step: one y plane of one column.  grid (ncols, N2, nk): the blocks resident
// together share the y plane of Theta V in L2.
// LDS: X [nbz][n1+1] (kz rows, x), Z [n3][xc+1] (a chunk of xc x columns), twiddles.
template <int L1, int L3>
__global__ __launch_bounds__(FFT_NT) void k_rb_xz(const Grid g, const FftKArgs ka, int ncols, int xc,
                                                  const double *__restrict__ thv) {
  extern __shared__ double2 sm[];
  const int col = blockIdx.x, y = blockIdx.y, kk = blockIdx.z;
  const int n1 = L1 > 0 ? L1 : g.n1, n2 = g.n2, n3 = L3 > 0 ? L3 : g.n3;
  const int bx = g.bx, nbx = g.nbx, bz = g.bz, nbz = g.nbz;
  const int xp = n1 + 1, zp = xc + 1;
  double2 *X = sm;
  double2 *Z = X + nbz * xp;
  double2 *tw1 = Z + n3 * zp;
  double2 *tw3 = tw1 + n1;
  load_tw(tw1, g.tw1, n1);
  load_tw(tw3, g.tw3, n3);
  const long long csz = (long long)nbz * n2 * nbx;
  const double2 *in = ka.slab_in[kk] + (long long)col * csz + (long long)y * nbx;
  double2 *out = ka.slab_out[kk] + (long long)col * csz + (long long)y * nbx;
  const long long rs = (long long)n2 * nbx;  // kz stride of the box arrays
  for (int i = threadIdx.x; i < nbz * n1; i += blockDim.x) {
    const int p = i / n1, x = i - p * n1;
    const int b = box_of(x, n1, bx);
    X[p * xp + x] = (b >= 0) ? in[p * rs + b] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  fft_block<1, L1>(X, LinesUniform{0, xp}, nbz, 1, g.p1, tw1);  // inverse along x
  const long long plane = (long long)n1 * n2;
  for (int x0 = 0; x0 < n1; x0 += xc) {
    const int nc = (n1 - x0) < xc ? (n1 - x0) : xc;
    for (int i = threadIdx.x; i < n3 * xc; i += blockDim.x) {
      const int z = i / xc, cc = i - z * xc;
      const int kz = z <= bz ? z : z - n3;
      Z[z * zp + cc] = (cc < nc && kz >= -bz && kz <= bz) ? X[(kz + bz) * xp + x0 + cc] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    fft_block<1, L3>(Z, LinesUniform{0, 1}, nc, zp, g.p3, tw3);  // inverse along z
    for (int i = threadIdx.x; i < n3 * nc; i += blockDim.x) {
      const int z = i / nc, cc = i - z * nc;
      Z[z * zp + cc] = cscale(Z[z * zp + cc], thv[(long long)z * plane + (long long)y * n1 + x0 + cc]);
    }
    __syncthreads();
    fft_block<-1, L3>(Z, LinesUniform{0, 1}, nc, zp, g.p3, tw3);  // forward along z
    for (int i = threadIdx.x; i < nbz * nc; i += blockDim.x) {
      const int p = i / nc, cc = i - p * nc;
      const int kz = p - bz;
      X[p * xp + x0 + cc] = Z[(kz < 0 ? kz + n3 : kz) * zp + cc];
    }
    __syncthreads();
  }
  fft_block<-1, L1>(X, LinesUniform{0, xp}, nbz, 1, g.p1, tw1);  // forward along x
  for (int i = threadIdx.x; i < nbz * nbx; i += blockDim.x) {
    const int p = i / nbx, b = i - p * nbx;
    const int kx = b - bx;
    out[p * rs + b] = X[p * xp + (kx < 0 ? kx + n1 : kx)];
  }
}

// Step: forward y transforms of one kz plane of the box array and the sphere
// read-out Y[g, col] = (1/N) value.  grid (nbz, ncols, nk).
template <int L2, class T>
__global__ __launch_bounds__(FFT_NT) void k_rb_y(const Grid g, const FftKArgs ka, int ncols) {
  extern __shared__ double2 sm_raw[];
  T *sm = reinterpret_cast<T *>(sm_raw);
  const int pz = blockIdx.x, col = blockIdx.y, kk = blockIdx.z;
  const int n1 = g.n1, n2 = L2 > 0 ? L2 : g.n2;
  const int bx = g.bx, nbx = g.nbx;
  const int bp = n2 + 1;
  T *bxc = sm;
  T *tw2 = bxc + nbx * bp;
  load_tw(tw2, g.tw2, n2);
  const KSphere &sp = ka.sph[kk];
  const FwdOut &fo = ka.out[kk];
  const long long csz = (long long)g.nbz * n2 * nbx;
  const T *src = reinterpret_cast<const T *>(ka.slab_in[kk]) + (long long)col * csz + (long long)pz * n2 * nbx;
  stage8<T>(
      n2 * nbx, [&](int i) { return src[i]; }, [&](int i, T x) { bxc[(i % nbx) * bp + i / nbx] = x; });
  __syncthreads();
  fft_block<-1, L2>(bxc, LinesUniform{0, bp}, nbx, 1, g.p2, tw2);
  const double inv_n = 1.0 / ((double)n1 * n2 * g.n3);
  const int p0 = sp.plane_ptr[pz], p1 = sp.plane_ptr[pz + 1];
  for (int i = p0 + threadIdx.x; i < p1; i += blockDim.x) {
    const int xy = sp.pts_xy[i];
    const int yy = xy / g.d1, x = xy - yy * g.d1;
    const int yr = yy <= g.by ? yy : yy - g.d2 + n2;
    const double2 val = cscale(to_d2(bxc[box_of(x, g.d1, bx) * bp + yr]), inv_n);
    if (fo.o0f) fo.o0f[i + (long long)col * fo.ld0] = make_float2((float)val.x, (float)val.y);
    else fo.o0[i + (long long)col * fo.ld0] = val;
  }
}

// ---------------------------------------------------------------------------
// Rebuild path, two-factor register transforms.  A line of length N = F1 * F2
// is transformed by F2 lanes holding F1 values each, one exchange through a
// per-wave LDS scratch, then F1 lanes holding F2 values each (w_M = exp(DIR 2 pi i/M)):
//   inverse, input n = F2 n1 + n2, output k = k1 + F1 k2:
//     X[k1 + F1 k2] = sum_n2 w_F2^(n2 k2) w_N^(n2 k1) sum_n1 w_F1^(n1 k1) x[F2 n1 + n2]
//   forward, input z = a + F1 b, output m = F2 c + d:
//     Q[F2 c + d] = sum_a w_F1^(a c) w_N^(a d) sum_b w_F2^(b d) P[a + F1 b]
// The inverse's output layout (lane k1 holds k1 + F1 k2) is the forward's input
// layout, so a z column stays in registers from its inverse transform through
// the Theta V product to its forward transform.  Lines live inside one wave
// (G = max(F1, F2) lanes each); the exchange needs no block barrier.
// ---------------------------------------------------------------------------
template <int N, int F1, int F2>
struct Two {
  static_assert(F1 * F2 == N, "two-factor length");
  static constexpr int G = F1 > F2 ? F1 : F2;             // lanes per line
  static constexpr int LPW = 64 / G;                      // lines per wave
  static constexpr int P = (G % 2) ? G : G + 1;           // odd pitch of the exchange rows
  static constexpr int LS = G * P + ((9 - (G * P) % 8) % 8);  // line stride, = 1 mod 8
};

// z columns per wave and pass of k_rb_xz4: up to 8, as many lines as fit a wave
constexpr int rb_lz(int lpw) { return lpw < 8 ? lpw : 8; }
constexpr int rb_pitch(int n) { return n + ((9 - n % 8) % 8); }  // >= n, = 1 mod 8

__device__ __forceinline__ void wave_fence() { __atomic_signal_fence(__ATOMIC_SEQ_CST); }

// On an exact rebuild grid (N >= 4 b + 1, so b <= (N - 1) / 4) the inputs of a
// line at frequencies b < n < N - b are zero and its outputs there are never
// read.  With n = F2 n1 + r (r < F2, the lane's role) that holds for every lane
// when n1 is in [zr_lo, zr_hi]: those register values are zero before the first
// pass of an inverse transform and unused after the last pass of a forward one.
template <int N, int F2>
constexpr int zr_lo() { return ((N - 1) / 4 + F2) / F2; }
template <int N, int F2>
constexpr int zr_hi() { return (N - (N - 1) / 4 - F2) / F2; }
// first pass of a line whose inputs LO..HI are zero
template <int R, int DIR, int LO, int HI, class T>
__device__ __forceinline__ void dft_first(T *v);

// base twiddle w_N^role (inverse sign) of this lane
__device__ __forceinline__ double2 role_twiddle(int role, int n) {
  double sv, cv;
  sincospi(2.0 * role / n, &sv, &cv);
  return make_double2(cv, sv);
}

// v[j] *= w^j, j = 1 .. R-1 (powers by repeated products)
template <int R, class T>
__device__ __forceinline__ void twiddle_powers(T *v, T w) {
  T p = w;
#pragma unroll
  for (int j = 1; j < R; ++j) {
    v[j] = cmul(v[j], p);
    if (j + 1 < R) p = cmul(p, w);
  }
}

// v[j] *= t[j] (DIR = -1) or conj(t[j]) (DIR = +1), j = 1 .. R-1: the twiddles of
// one lane from its table of exp(-2 pi i role j / N)
template <int R, int DIR, class T>
__device__ __forceinline__ void twiddle_tab(T *v, const T *t) {
#pragma unroll
  for (int j = 1; j < R; ++j) v[j] = cmul(v[j], DIR < 0 ? t[j] : cconj(t[j]));
}

// LDS layout of k_rb_xz4.  On 64-point lines (8 x 8) the exchange slots of
// value (i, j) of a line's 8 x 8 block are i 8 + (j ^ i) (XOR swizzle), the
// rows have pitch 66 (complex128) or 68 (complex64) and the two rows a 16-lane
// group touches are r and r + 4, and the z scratch lines are 72 apart: every
// access of the kernel then hits distinct LDS banks (16-lane groups of 16-byte
// accesses).  Other lengths keep odd pitches.
template <int NX, int X1, int NZ, int Z1>
constexpr bool xz4_swz() { return NX == 64 && X1 == 8 && NZ == 64 && Z1 == 8; }
template <int NX, int X1, int NZ, int Z1, class T>
constexpr int xz4_rx() { return xz4_swz<NX, X1, NZ, Z1>() ? (sizeof(T) == 16 ? 66 : 68) : rb_pitch(NX); }
// z-line exchange pitches of the general lengths: slots (i, j) at i P1 + j in the
// first exchange (rows i < Z2, columns j < Z1), i P2 + j in the second (rows
// i < Z1, columns j < Z2), lines LS apart.  For 108 = 12 x 9 (12 lanes per line,
// five lines per wave, 8-byte slots) P1 = 13, P2 = 9 and LS = 117 (the smallest
// that holds both) keep a complex128 block of four such waves within half the
// LDS of a CU; a bank model of all the kernel's LDS accesses (64 banks of 4
// bytes, 16-byte accesses 16 lanes per cycle, 8-byte ones 32) gives 1,296
// conflict cycles per block against 4,986 measured for the odd pitch 13 with
// lines 161 apart.  Other lengths keep the odd pitch of Two.
template <int NZ, int Z1>
struct XchPitch {
  using TZ = Two<NZ, Z1, NZ / Z1>;
  static constexpr bool TUNED = (NZ == 108);
  static constexpr int P1 = TZ::P;
  static constexpr int P2 = TUNED ? NZ / Z1 : TZ::P;
  static constexpr int need = ((NZ / Z1 - 1) * P1 + Z1) > ((Z1 - 1) * P2 + NZ / Z1) ? ((NZ / Z1 - 1) * P1 + Z1)
                                                                                    : ((Z1 - 1) * P2 + NZ / Z1);
  static constexpr int LS = TUNED ? need + 1 : TZ::LS;
};
template <int NX, int X1, int NZ, int Z1>
constexpr int xz4_ls() { return xz4_swz<NX, X1, NZ, Z1>() ? 72 : XchPitch<NZ, Z1>::LS; }
// exchange slot of (i, j) in a block of rows of length `pitch` (swizzled or plain)
template <bool SWZ>
__device__ __forceinline__ int xslot(int i, int j, int pitch) { return SWZ ? i * 8 + (j ^ i) : i * pitch + j; }
// complex128 on the swizzled 8 x 8 layout: the z lines exchange their real and
// imaginary parts one after the other through a scratch of doubles (lines 72
// doubles apart, again distinct banks for every 32-lane group of 8-byte
// accesses), half the LDS of a complex scratch: three blocks fit a CU
// Every complex128 instance exchanges its z lines this way (the 8 x 8 layout
// through xch8_split, the others through xch_split): half the LDS of a complex
// scratch, so that two blocks of the 72 x 108 kernel (8 waves) share a CU.
template <int NX, int X1, int NZ, int Z1, class T>
constexpr bool xz4_split() { return sizeof(T) == 16; }
// LDS bytes of k_rb_xz4 (rows, then NW x LZ z-line scratch)
template <int NX, int X1, int NZ, int Z1, class T>
constexpr size_t xz4_lds(int nbz, int nw, int lz) {
  return (size_t)nbz * xz4_rx<NX, X1, NZ, Z1, T>() * sizeof(T) +
         (size_t)nw * lz * xz4_ls<NX, X1, NZ, Z1>() * (xz4_split<NX, X1, NZ, Z1, T>() ? sizeof(double) : sizeof(T));
}

// 8 x 8 transpose of one z line through its scratch sd (doubles, slot xslot<true>):
// lane r holds in[k] = value (r, k) and receives out[q] = value (q, r); the real
// parts pass first, then the imaginary parts through the same slots (LDS
// operations of one wave complete in order, so no wait is needed between them)
__device__ __forceinline__ void xch8_split(double *sd, int r, const double2 (&in)[8], double2 (&out)[8]) {
#pragma unroll
  for (int k = 0; k < 8; ++k) sd[xslot<true>(r, k, 8)] = in[k].x;
  wave_fence();
#pragma unroll
  for (int q = 0; q < 8; ++q) out[q].x = sd[xslot<true>(q, r, 8)];
  wave_fence();
#pragma unroll
  for (int k = 0; k < 8; ++k) sd[xslot<true>(r, k, 8)] = in[k].y;
  wave_fence();
#pragma unroll
  for (int q = 0; q < 8; ++q) out[q].y = sd[xslot<true>(q, r, 8)];
  wave_fence();
}

// Exchange of one z line of a two-factor transform through a scratch of doubles
// sd (slots i P + j): lanes with `put` write vin[k] to slot (r, k), k < RI,
// lanes with `get` read vout[q] = slot (q, r), q < RO; the real parts pass
// first, then the imaginary parts (LDS operations of one wave complete in order).
template <int RI, int RO>
__device__ __forceinline__ void xch_split(double *sd, int r, int P, bool put, bool get, const double2 (&vin)[RI],
                                          double2 (&vout)[RO]) {
  if (put)
#pragma unroll
    for (int k = 0; k < RI; ++k) sd[r * P + k] = vin[k].x;
  wave_fence();
  if (get)
#pragma unroll
    for (int q = 0; q < RO; ++q) vout[q].x = sd[q * P + r];
  wave_fence();
  if (put)
#pragma unroll
    for (int k = 0; k < RI; ++k) sd[r * P + k] = vin[k].y;
  wave_fence();
  if (get)
#pragma unroll
    for (int q = 0; q < RO; ++q) vout[q].y = sd[q * P + r];
  wave_fence();
}

// Same transforms with NW waves per block: an x row exchanges in place through
// its own RX slots (value (k1, n2) at slot k1 F2 + n2, odd stride across lanes);
// the z columns exchange through a per-wave scratch of LZ lines.
// T: element type (double2, or float2 for the FP32 residual); thp in its real type.
template <int R, int DIR, int LO, int HI, class T>
__device__ __forceinline__ void dft_first(T *v) {
  if constexpr (R == 8 && LO == 2 && HI == 5) dft8_z2345<DIR>(v);
  else if constexpr (R == 12 && LO == 3 && HI == 8) dft12_z3to8<DIR>(v);
  else dft_reg<R, DIR>(v);
}

// PR: the box fits the exact-grid bound on both axes (4 b + 1 <= N), so the
// known-zero inputs and unread outputs of every line are dropped at compile
// time (the 64-point instance always does, under its own b <= 15 check).
template <int NX, int X1, int X2, int NZ, int Z1, int Z2, int NW, int LZ, class T, bool PR>
__global__ __launch_bounds__(NW * 64) void k_rb_xz4(const Grid g, const FftKArgs ka, int ncols,
                                                   const typename CT<T>::R *__restrict__ thp) {
  using RT = typename CT<T>::R;
  using TX = Two<NX, X1, X2>;
  using TZ = Two<NZ, Z1, Z2>;
  using XP = XchPitch<NZ, Z1>;
  static_assert(LZ <= TZ::LPW, "z lines per wave");
  constexpr bool SWZ = xz4_swz<NX, X1, NZ, Z1>();
  constexpr int RX = xz4_rx<NX, X1, NZ, Z1, T>();
  constexpr int LS = xz4_ls<NX, X1, NZ, Z1>();
  constexpr bool SPLIT = SWZ && sizeof(T) == 16;   // the 8 x 8 split exchange
  constexpr bool SPLITG = !SWZ && sizeof(T) == 16;  // the general split exchange
  constexpr bool PX = SWZ || PR;                    // dropped x and z values
  constexpr int XLO = zr_lo<NX, X2>(), XHI = zr_hi<NX, X2>();
  constexpr int ZLO = zr_lo<NZ, Z2>(), ZHI = zr_hi<NZ, Z2>();
  static_assert(!SWZ || (XLO == 2 && XHI == 5 && ZLO == 2 && ZHI == 5), "64-point pruning range");
  extern __shared__ double2 sm_raw[];
  T *sm = reinterpret_cast<T *>(sm_raw);
  const int col = blockIdx.x, y = blockIdx.y, kk = blockIdx.z;
  const int n2 = g.n2, bx = g.bx, nbx = g.nbx, bz = g.bz, nbz = g.nbz;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  T *R = sm;
  T *scr = sm + nbz * RX + wave * (LZ * LS);  // complex scratch (!SPLIT)
  double *scd = reinterpret_cast<double *>(sm + nbz * RX) + wave * (LZ * LS);  // SPLIT
  const long long csz = (long long)nbz * n2 * nbx;
  const long long rs = (long long)n2 * nbx;  // kz stride of the box arrays
  const T *in = reinterpret_cast<const T *>(ka.slab_in[kk]) + (long long)col * csz + (long long)y * nbx;
  T *out = reinterpret_cast<T *>(ka.slab_out[kk]) + (long long)col * csz + (long long)y * nbx;
  const int lx = lane / TX::G, rx = lane - lx * TX::G;
  const int lz = lane / TZ::G, rz = lane - lz * TZ::G;
  // row of line lx within a wave's group of LPW rows (SWZ: a 16-lane group takes rows r, r + 4)
  const int lxr = SWZ ? ((lx >> 1) | ((lx & 1) << 2)) : lx;
  // SWZ (x and z 8 x 8, rx == rz): this lane's twiddles exp(-2 pi i rx j / 64), j < 8,
  // shared by the four two-factor passes
  T twt[8];
  if constexpr (SWZ) {
#pragma unroll
    for (int j = 0; j < 8; ++j) twt[j] = CT<T>::from(g.tw1[(rx * j) & 63]);
  }

  // phase 1: inverse x transforms of the box rows, in place in R
  {
    const T w = CT<T>::from(cconj(g.tw1[rx < NX ? rx : 0]));
    for (int r0 = wave * TX::LPW; r0 < nbz; r0 += NW * TX::LPW) {
      const int r = r0 + lxr;
      const bool on = lx < TX::LPW && r < nbz;
      T *row = R + r * RX;
      if (on && rx < X2) {
        T v[X1];
#pragma unroll
        for (int n1 = 0; n1 < X1; ++n1) {
          if (PX && n1 >= XLO && n1 <= XHI) {  // b < |freq|: zero (dropped by the first pass)
            v[n1] = CT<T>::mk(0, 0);
            continue;
          }
          const int n = X2 * n1 + rx;
          const int kx = n <= bx ? n : n - NX;
          v[n1] = (n <= bx || n >= NX - bx) ? in[r * rs + kx + bx] : CT<T>::mk(0, 0);
        }
        if constexpr (SWZ) {
          dft8_z2345<1>(v);
          twiddle_tab<X1, 1>(v, twt);
        } else {
          if constexpr (PR) dft_first<X1, 1, XLO, XHI>(v);
          else dft_reg<X1, 1>(v);
          twiddle_powers<X1>(v, w);
        }
#pragma unroll
        for (int k1 = 0; k1 < X1; ++k1) row[xslot<SWZ>(k1, rx, X2)] = v[k1];
      }
      wave_fence();
      if (on && rx < X1) {
        T u[X2];
#pragma unroll
        for (int q = 0; q < X2; ++q) u[q] = row[xslot<SWZ>(rx, q, X2)];
        dft_reg<X2, 1>(u);
        wave_fence();
#pragma unroll
        for (int k2 = 0; k2 < X2; ++k2) row[rx + X1 * k2] = u[k2];
      }
      wave_fence();
    }
  }
  __syncthreads();

  // phase 2: z columns, inverse -> product -> forward, in place in the box rows
  {
    const T w = CT<T>::from(cconj(g.tw3[rz < NZ ? rz : 0])), wc = cconj(w);
    for (int x0 = wave * LZ; x0 < NX; x0 += NW * LZ) {
      const int x = x0 + lz;
      const bool on = lz < LZ && x < NX;
      T *sl = scr + lz * LS;
      // Theta V of this column (used after the inverse): loads issued first
      RT t[Z2];
#pragma unroll
      for (int k2 = 0; k2 < Z2; ++k2)
        t[k2] = thp[(((long long)y * Z2 + k2) * NX + (x < NX ? x : NX - 1)) * Z1 + (rz < Z1 ? rz : 0)];
      if constexpr (SPLIT) {  // 8 x 8, complex128: the same transforms, split exchanges
        if (on) {
          double2 v[8], u[8];
#pragma unroll
          for (int n1 = 0; n1 < 8; ++n1) {
            if (n1 >= 2 && n1 <= 5) {
              v[n1] = make_double2(0.0, 0.0);
              continue;
            }
            const int n = 8 * n1 + rz;
            const int row = n <= bz ? n + bz : n - NZ + bz;
            v[n1] = (n <= bz || n >= NZ - bz) ? R[row * RX + x] : make_double2(0.0, 0.0);
          }
          dft8_z2345<1>(v);
          twiddle_tab<8, 1>(v, twt);
          double *sd = scd + lz * LS;
          xch8_split(sd, rz, v, u);
          dft_reg<8, 1>(u);
#pragma unroll
          for (int k2 = 0; k2 < 8; ++k2) u[k2] = cscale(u[k2], t[k2]);
          dft_reg<8, -1>(u);
          twiddle_tab<8, -1>(u, twt);
          xch8_split(sd, rz, u, v);
          dft_reg<8, -1>(v);
#pragma unroll
          for (int c = 0; c < 8; ++c) {
            if (c >= 2 && c <= 5) continue;
            const int m = 8 * c + rz;
            if (m <= bz || m >= NZ - bz) R[(m <= bz ? m + bz : m - NZ + bz) * RX + x] = v[c];
          }
        }
        wave_fence();
        continue;
      }
      if constexpr (SPLITG) {  // complex128, general lengths: split exchanges through doubles
        double *sd = scd + lz * LS;
        double2 v[Z1], u[Z2];
        if (on && rz < Z2) {
#pragma unroll
          for (int n1 = 0; n1 < Z1; ++n1) {
            if (PR && n1 >= ZLO && n1 <= ZHI) {
              v[n1] = make_double2(0.0, 0.0);
              continue;
            }
            const int n = Z2 * n1 + rz;
            const int row = n <= bz ? n + bz : n - NZ + bz;
            v[n1] = (n <= bz || n >= NZ - bz) ? R[row * RX + x] : make_double2(0.0, 0.0);
          }
          if constexpr (PR) dft_first<Z1, 1, ZLO, ZHI>(v);
          else dft_reg<Z1, 1>(v);
          twiddle_powers<Z1>(v, w);
        }
        xch_split<Z1, Z2>(sd, rz, XP::P1, on && rz < Z2, on && rz < Z1, v, u);
        if (on && rz < Z1) {
          dft_reg<Z2, 1>(u);
#pragma unroll
          for (int k2 = 0; k2 < Z2; ++k2) u[k2] = cscale(u[k2], t[k2]);
          dft_reg<Z2, -1>(u);
          twiddle_powers<Z2>(u, wc);
        }
        xch_split<Z2, Z1>(sd, rz, XP::P2, on && rz < Z1, on && rz < Z2, u, v);
        if (on && rz < Z2) {
          dft_reg<Z1, -1>(v);
#pragma unroll
          for (int c = 0; c < Z1; ++c) {
            if (PR && c >= ZLO && c <= ZHI) continue;  // never read: not computed
            const int m = Z2 * c + rz;
            if (m <= bz || m >= NZ - bz) R[(m <= bz ? m + bz : m - NZ + bz) * RX + x] = v[c];
          }
        }
        wave_fence();
        continue;
      }
      if (on && rz < Z2) {
        T v[Z1];
#pragma unroll
        for (int n1 = 0; n1 < Z1; ++n1) {
          if (PX && n1 >= ZLO && n1 <= ZHI) {
            v[n1] = CT<T>::mk(0, 0);
            continue;
          }
          const int n = Z2 * n1 + rz;
          const int row = n <= bz ? n + bz : n - NZ + bz;
          v[n1] = (n <= bz || n >= NZ - bz) ? R[row * RX + x] : CT<T>::mk(0, 0);
        }
        if constexpr (SWZ) {
          dft8_z2345<1>(v);
          twiddle_tab<Z1, 1>(v, twt);
        } else {
          if constexpr (PR) dft_first<Z1, 1, ZLO, ZHI>(v);
          else dft_reg<Z1, 1>(v);
          twiddle_powers<Z1>(v, w);
        }
#pragma unroll
        for (int k1 = 0; k1 < Z1; ++k1) sl[xslot<SWZ>(rz, k1, XP::P1)] = v[k1];
      }
      wave_fence();
      if (on && rz < Z1) {
        T u[Z2];
#pragma unroll
        for (int q = 0; q < Z2; ++q) u[q] = sl[xslot<SWZ>(q, rz, XP::P1)];
        dft_reg<Z2, 1>(u);
#pragma unroll
        for (int k2 = 0; k2 < Z2; ++k2) u[k2] = cscale(u[k2], t[k2]);
        dft_reg<Z2, -1>(u);
        if constexpr (SWZ) twiddle_tab<Z2, -1>(u, twt);
        else twiddle_powers<Z2>(u, wc);
        wave_fence();
#pragma unroll
        for (int d = 0; d < Z2; ++d) sl[xslot<SWZ>(rz, d, XP::P2)] = u[d];
      }
      wave_fence();
      if (on && rz < Z2) {
        T v[Z1];
#pragma unroll
        for (int a = 0; a < Z1; ++a) v[a] = sl[xslot<SWZ>(a, rz, XP::P2)];
        dft_reg<Z1, -1>(v);
#pragma unroll
        for (int c = 0; c < Z1; ++c) {
          if (PX && c >= ZLO && c <= ZHI) continue;  // b < |freq|: never needed
          const int m = Z2 * c + rz;
          if (m <= bz || m >= NZ - bz) R[(m <= bz ? m + bz : m - NZ + bz) * RX + x] = v[c];
        }
      }
      wave_fence();
    }
  }
  __syncthreads();

  // phase 3: forward x transforms of the box rows, box columns out
  {
    const T wc = CT<T>::from(g.tw1[rx < NX ? rx : 0]);
    for (int r0 = wave * TX::LPW; r0 < nbz; r0 += NW * TX::LPW) {
      const int r = r0 + lxr;
      const bool on = lx < TX::LPW && r < nbz;
      T *row = R + r * RX;
      if (on && rx < X1) {
        T u[X2];
#pragma unroll
        for (int b = 0; b < X2; ++b) u[b] = row[rx + X1 * b];
        dft_reg<X2, -1>(u);
        if constexpr (SWZ) twiddle_tab<X2, -1>(u, twt);
        else twiddle_powers<X2>(u, wc);
        wave_fence();
#pragma unroll
        for (int d = 0; d < X2; ++d) row[xslot<SWZ>(rx, d, X2)] = u[d];
      }
      wave_fence();
      if (on && rx < X2) {
        T v[X1];
#pragma unroll
        for (int a = 0; a < X1; ++a) v[a] = row[xslot<SWZ>(a, rx, X2)];
        dft_reg<X1, -1>(v);
#pragma unroll
        for (int c = 0; c < X1; ++c) {
          if (PX && c >= XLO && c <= XHI) continue;
          const int m = X2 * c + rx;
          if (m <= bx || m >= NX - bx) out[r * rs + (m <= bx ? m : m - NX) + bx] = v[c];
        }
      }
      wave_fence();
    }
  }
}

// ---------------------------------------------------------------------------
// Line pass of the apply along z with the two-factor register transforms of the
// rebuild (NZ = Z1 x Z2, the box within the exact-grid bound 4 bz + 1 <= NZ): a
// wave takes LZ lines at consecutive (x, y) positions, TZ::G lanes each.  Per
// input field: the inverse line transform (known-zero inputs dropped), the
// products with Theta (and Theta V) held in registers, the forward transforms
// (unread outputs not computed) and the box values out, with the z lines
// exchanged through a per-wave scratch of doubles (real parts, then imaginary
// parts).  Fields as k_lines: MODE_V psi -> m psi (m = thv); otherwise psi,
// pi_x, pi_y, pi_z -> Theta psi, Theta V psi, Theta pi_x psi, Theta pi_y psi,
// Theta pi_z psi.  Four waves per block.
// ---------------------------------------------------------------------------
template <int NZ, int Z1, bool VMODE>
__global__ __launch_bounds__(256) void k_lines_reg(const Grid g, const FftKArgs ka, int ncols,
                                                   const double *__restrict__ thv) {
  constexpr int Z2 = NZ / Z1;
  using TZ = Two<NZ, Z1, Z2>;
  using XP = XchPitch<NZ, Z1>;
  constexpr int LZ = rb_lz(TZ::LPW);
  constexpr int ZLO = zr_lo<NZ, Z2>(), ZHI = zr_hi<NZ, Z2>();
  extern __shared__ double2 sm_raw[];
  const int col = blockIdx.y, kk = blockIdx.z;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lz = lane / TZ::G, rz = lane - lz * TZ::G;
  const long long plane = (long long)g.n1 * g.n2;
  const int bz = g.bz, nbz = g.nbz;
  const long long pos = ((long long)blockIdx.x * 4 + wave) * LZ + lz;
  const bool on = lz < LZ && pos < plane;
  const long long pc = on ? pos : 0;  // clamped position (loads of idle lanes stay in bounds)
  double *sd = reinterpret_cast<double *>(sm_raw) + (long long)(wave * LZ + (lz < LZ ? lz : 0)) * XP::LS;
  const long long fstride = (long long)ncols * nbz * plane;
  const double2 *in = ka.slab_in[kk] + (long long)col * nbz * plane + pc;
  double2 *out = ka.slab_out[kk] + (long long)col * nbz * plane + pc;
  const double2 w = cconj(g.tw3[rz < NZ ? rz : 0]), wc = cconj(w);
  // the multipliers at z = rz + Z1 k2, the layout of a line after its inverse transform
  double m0[Z2], m1[Z2];
  {
    const int r = rz < Z1 ? rz : 0;
#pragma unroll
    for (int k2 = 0; k2 < Z2; ++k2) {
      const long long e = (long long)(r + Z1 * k2) * plane + pc;
      m0[k2] = VMODE ? thv[e] : g.theta[e];
      m1[k2] = VMODE ? 0.0 : thv[e];
    }
  }
  // inverse transform of input field f into u (lanes rz < Z1)
  auto inverse = [&](int f, double2 (&u)[Z2]) {
    double2 v[Z1];
    if (on && rz < Z2) {
      const double2 *src = in + (long long)f * fstride;
#pragma unroll
      for (int n1 = 0; n1 < Z1; ++n1) {
        if (n1 >= ZLO && n1 <= ZHI) {
          v[n1] = make_double2(0.0, 0.0);
          continue;
        }
        const int n = Z2 * n1 + rz;
        const int row = n <= bz ? n + bz : n - NZ + bz;
        v[n1] = (n <= bz || n >= NZ - bz) ? src[(long long)row * plane] : make_double2(0.0, 0.0);
      }
      dft_first<Z1, 1, ZLO, ZHI>(v);
      twiddle_powers<Z1>(v, w);
    }
    xch_split<Z1, Z2>(sd, rz, XP::P1, on && rz < Z2, on && rz < Z1, v, u);
    if (on && rz < Z1) dft_reg<Z2, 1>(u);
  };
  // forward transform of u times m into output field o
  auto forward = [&](const double2 (&u)[Z2], const double (&m)[Z2], int o) {
    double2 p[Z2], q[Z1];
    if (on && rz < Z1) {
#pragma unroll
      for (int k2 = 0; k2 < Z2; ++k2) p[k2] = cscale(u[k2], m[k2]);
      dft_reg<Z2, -1>(p);
      twiddle_powers<Z2>(p, wc);
    }
    xch_split<Z2, Z1>(sd, rz, XP::P2, on && rz < Z1, on && rz < Z2, p, q);
    if (on && rz < Z2) {
      dft_reg<Z1, -1>(q);
      double2 *dst = out + (long long)o * fstride;
#pragma unroll
      for (int c = 0; c < Z1; ++c) {
        if (c >= ZLO && c <= ZHI) continue;  // b < |freq|: never read
        const int mm = Z2 * c + rz;
        if (mm <= bz || mm >= NZ - bz) dst[(long long)(mm <= bz ? mm + bz : mm - NZ + bz) * plane] = q[c];
      }
    }
  };
  double2 u[Z2];
  inverse(0, u);
  forward(u, m0, 0);
  if constexpr (!VMODE) {
    forward(u, m1, 1);
#pragma unroll 1
    for (int f = 1; f <= 3; ++f) {
      inverse(f, u);
      forward(u, m0, f + 1);
    }
  }
}

// ---------------------------------------------------------------------------
// Plane passes of the apply with the two-factor register transforms, for square
// planes N1 = N2 = N = F1 F2 (72 = 8 x 9, 64 = 8 x 8) with the box within the
// exact-grid bound (4 b + 1 <= N on x and y).  One block (four waves) per (kz
// plane, column), as k_inv_plane / k_fwd_plane, with the same slab layout and
// the same sums up to rounding order.  A line takes Two<N>::G lanes (a lane of
// role r holds the values r + F2 n1 before the first pass, r + F1 k2 after the
// second); the box columns B[kx][y] (pitch RP = rb_pitch(N)) stay in LDS and
// exchange in place, the x rows exchange through a per-wave scratch of doubles
// (real parts, then imaginary parts).  Known-zero inputs (|k| > b) are dropped
// before the first pass, outputs outside the box are never computed.  The
// plane's sphere points are read once per block into registers (PLANE_PPT per
// thread, two for the four outputs of MODE_TVPS; points beyond that times 256
// go through global memory per field), and the forward pass keeps its outputs
// there across the fields.
// ---------------------------------------------------------------------------
constexpr int PLANE_PPT = 3;
template <int N>
constexpr size_t plane_reg_lds(int nbx) {
  using TT = Two<N, 8, N / 8>;
  return (size_t)nbx * rb_pitch(N) * sizeof(double2) + (size_t)4 * TT::LPW * TT::LS * sizeof(double);
}

// Inverse: sphere coefficients (times 1 or (G+k)_i, fields as k_inv_plane) ->
// box columns -> inverse y transforms in place -> per grid row y the inverse x
// transform from the box columns, written to the slab row.
template <int N>
__global__ __launch_bounds__(256) void k_inv_plane_reg(const Grid g, const FftKArgs ka, int ncols, int nfields) {
  constexpr int F1 = 8, F2 = N / F1;
  using TT = Two<N, F1, F2>;
  constexpr int G = TT::G, LPW = TT::LPW, RP = rb_pitch(N), P = TT::P, LS = TT::LS;
  constexpr int LO = zr_lo<N, F2>(), HI = zr_hi<N, F2>();
  extern __shared__ double2 sm_raw[];
  const int pz = blockIdx.x, col = blockIdx.y, kk = blockIdx.z;
  const int bx = g.bx, nbx = g.nbx;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane / G, r = lane - li * G;
  double2 *B = sm_raw;
  double *sd = reinterpret_cast<double *>(B + nbx * RP) + (wave * LPW + (li < LPW ? li : 0)) * LS;
  const KSphere &sp = ka.sph[kk];
  const InvIn in = ka.in[kk];
  const int p0 = sp.plane_ptr[pz], p1 = sp.plane_ptr[pz + 1];
  constexpr long long plane_sz = (long long)N * N;
  const long long fstride = (long long)ncols * g.nbz * plane_sz;
  double2 *out = ka.slab_out[kk] + ((long long)col * g.nbz + pz) * plane_sz;
  // this lane's twiddles exp(-2 pi i r j / N), j < F1 (used conjugated)
  double2 twt[F1];
#pragma unroll
  for (int j = 0; j < F1; ++j) twt[j] = g.tw1[(r * j) % N];
  // this thread's sphere points: coefficient, (G+k), LDS slot (-1: none)
  double2 pc[PLANE_PPT];
  double pk[PLANE_PPT][3];
  int ps[PLANE_PPT];
#pragma unroll
  for (int k = 0; k < PLANE_PPT; ++k) {
    const int i = p0 + threadIdx.x + k * (int)blockDim.x;
    ps[k] = -1;
    if (i < p1) {
      const int gi = sp.pts_g[i], xy = sp.pts_xy[i];
      const int y = xy / N, x = xy - y * N;
      ps[k] = box_of(x, N, bx) * RP + y;
      pc[k] = in.c[(long long)gi + (long long)col * in.ldc];
      if (nfields > 1)
#pragma unroll
        for (int d = 0; d < 3; ++d) pk[k][d] = sp.gk[3 * gi + d];
    }
  }
  for (int f = 0; f < nfields; ++f) {
    for (int i = threadIdx.x; i < nbx * RP; i += blockDim.x) B[i] = make_double2(0.0, 0.0);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PLANE_PPT; ++k)
      if (ps[k] >= 0) B[ps[k]] = f > 0 ? cscale(pc[k], pk[k][f - 1]) : pc[k];
    for (int i = p0 + threadIdx.x + PLANE_PPT * (int)blockDim.x; i < p1; i += blockDim.x) {
      const int gi = sp.pts_g[i], xy = sp.pts_xy[i];
      double2 c = in.c[(long long)gi + (long long)col * in.ldc];
      if (f > 0) c = cscale(c, sp.gk[3 * gi + (f - 1)]);
      const int y = xy / N, x = xy - y * N;
      B[box_of(x, N, bx) * RP + y] = c;
    }
    __syncthreads();
    // inverse y transforms of the box columns, in place
    for (int b0 = wave * LPW; b0 < nbx; b0 += 4 * LPW) {
      const int b = b0 + li;
      const bool on = li < LPW && b < nbx;
      double2 *row = B + (on ? b : 0) * RP;
      if (on && r < F2) {  // reads and writes only the slots r + F2 j of its line
        double2 v[F1];
#pragma unroll
        for (int n1 = 0; n1 < F1; ++n1) v[n1] = (n1 >= LO && n1 <= HI) ? make_double2(0.0, 0.0) : row[F2 * n1 + r];
        dft_first<F1, 1, LO, HI>(v);
        twiddle_tab<F1, 1>(v, twt);
#pragma unroll
        for (int k1 = 0; k1 < F1; ++k1) row[k1 * F2 + r] = v[k1];
      }
      wave_fence();
      if (on && r < F1) {
        double2 u[F2];
#pragma unroll
        for (int q = 0; q < F2; ++q) u[q] = row[r * F2 + q];
        dft_reg<F2, 1>(u);
        wave_fence();
#pragma unroll
        for (int k2 = 0; k2 < F2; ++k2) row[r + F1 * k2] = u[k2];
      }
      wave_fence();
    }
    __syncthreads();
    // inverse x transforms of the grid rows, from the box columns to the slab
    double2 *o = out + f * fstride;
    for (int y0 = wave * LPW; y0 < N; y0 += 4 * LPW) {
      const int y = y0 + li;
      const bool on = li < LPW && y < N;
      double2 v[F1], u[F2];
      if (on && r < F2) {
#pragma unroll
        for (int n1 = 0; n1 < F1; ++n1) {
          const int n = F2 * n1 + r;
          if (n1 >= LO && n1 <= HI) {
            v[n1] = make_double2(0.0, 0.0);
            continue;
          }
          v[n1] = (n <= bx || n >= N - bx) ? B[(n <= bx ? n + bx : n - N + bx) * RP + y] : make_double2(0.0, 0.0);
        }
        dft_first<F1, 1, LO, HI>(v);
        twiddle_tab<F1, 1>(v, twt);
      }
      xch_split<F1, F2>(sd, r, P, on && r < F2, on && r < F1, v, u);
      if (on && r < F1) {
        dft_reg<F2, 1>(u);
#pragma unroll
        for (int k2 = 0; k2 < F2; ++k2) o[(long long)y * N + r + F1 * k2] = u[k2];
      }
      wave_fence();
    }
    __syncthreads();  // the next field rewrites B
  }
}

// Inverse y transforms of the apply's box route: per (kz plane, column) the
// sphere coefficients of each input field (times 1 or (G+k)_i) into the box
// columns B[kx][y], their inverse y transforms in place (as k_inv_plane_reg),
// and the y image of the plane out: c[f][col][kz][y][kx] (the layout the x/z
// kernel reads, fstride values per field).  grid (nbz, ncols).
template <int N>
__global__ __launch_bounds__(256) void k_ap_inv_y(const Grid g, const FftKArgs ka, int ncols, int nfields) {
  constexpr int F1 = 8, F2 = N / F1;
  using TT = Two<N, F1, F2>;
  constexpr int G = TT::G, LPW = TT::LPW, RP = rb_pitch(N);
  constexpr int LO = zr_lo<N, F2>(), HI = zr_hi<N, F2>();
  extern __shared__ double2 sm_raw[];
  const int pz = blockIdx.x, col = blockIdx.y;
  const int bx = g.bx, nbx = g.nbx, nbz = g.nbz;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane / G, r = lane - li * G;
  double2 *B = sm_raw;
  const KSphere &sp = ka.sph[0];
  const InvIn in = ka.in[0];
  const int p0 = sp.plane_ptr[pz], p1 = sp.plane_ptr[pz + 1];
  const long long fstride = (long long)ncols * nbz * N * nbx;
  double2 *out = ka.slab_out[0] + ((long long)col * nbz + pz) * N * nbx;
  double2 twt[F1];
#pragma unroll
  for (int j = 0; j < F1; ++j) twt[j] = g.tw2[(r * j) % N];
  double2 pc[PLANE_PPT];
  double pk[PLANE_PPT][3];
  int ps[PLANE_PPT];
#pragma unroll
  for (int k = 0; k < PLANE_PPT; ++k) {
    const int i = p0 + threadIdx.x + k * (int)blockDim.x;
    ps[k] = -1;
    if (i < p1) {
      const int gi = sp.pts_g[i], xy = sp.pts_xy[i];
      const int y = xy / g.n1, x = xy - y * g.n1;
      ps[k] = box_of(x, g.n1, bx) * RP + y;
      pc[k] = in.c[(long long)gi + (long long)col * in.ldc];
      if (nfields > 1)
#pragma unroll
        for (int d = 0; d < 3; ++d) pk[k][d] = sp.gk[3 * gi + d];
    }
  }
  for (int f = 0; f < nfields; ++f) {
    for (int i = threadIdx.x; i < nbx * RP; i += blockDim.x) B[i] = make_double2(0.0, 0.0);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PLANE_PPT; ++k)
      if (ps[k] >= 0) B[ps[k]] = f > 0 ? cscale(pc[k], pk[k][f - 1]) : pc[k];
    for (int i = p0 + threadIdx.x + PLANE_PPT * (int)blockDim.x; i < p1; i += blockDim.x) {
      const int gi = sp.pts_g[i], xy = sp.pts_xy[i];
      double2 c = in.c[(long long)gi + (long long)col * in.ldc];
      if (f > 0) c = cscale(c, sp.gk[3 * gi + (f - 1)]);
      const int y = xy / g.n1, x = xy - y * g.n1;
      B[box_of(x, g.n1, bx) * RP + y] = c;
    }
    __syncthreads();
    for (int b0 = wave * LPW; b0 < nbx; b0 += 4 * LPW) {
      const int b = b0 + li;
      const bool on = li < LPW && b < nbx;
      double2 *row = B + (on ? b : 0) * RP;
      if (on && r < F2) {  // reads and writes only the slots r + F2 j of its line
        double2 v[F1];
#pragma unroll
        for (int n1 = 0; n1 < F1; ++n1) v[n1] = (n1 >= LO && n1 <= HI) ? make_double2(0.0, 0.0) : row[F2 * n1 + r];
        dft_first<F1, 1, LO, HI>(v);
        twiddle_tab<F1, 1>(v, twt);
#pragma unroll
        for (int k1 = 0; k1 < F1; ++k1) row[k1 * F2 + r] = v[k1];
      }
      wave_fence();
      if (on && r < F1) {
        double2 u[F2];
#pragma unroll
        for (int q = 0; q < F2; ++q) u[q] = row[r * F2 + q];
        dft_reg<F2, 1>(u);
        wave_fence();
#pragma unroll
        for (int k2 = 0; k2 < F2; ++k2) row[r + F1 * k2] = u[k2];
      }
      wave_fence();
    }
    __syncthreads();
    double2 *o = out + f * fstride;
    for (int i = threadIdx.x; i < N * nbx; i += blockDim.x) {
      const int y = i / nbx, b = i - y * nbx;
      o[i] = B[b * RP + y];
    }
    __syncthreads();  // the next field rewrites B
  }
}

// The forward pass's outputs of one sphere point, accumulated over the fields
// in the order of fwd_out_point (the same sums), stored after the last field.
template <int MODE>
struct FwdAcc {
  double2 a0, a1, a2, a3;
  __device__ __forceinline__ void add(int f, double2 val, const double *gk, double alpha_a, double beta_a) {
    if constexpr (MODE == FFT_MODE_V) {
      a0 = val;
    } else if constexpr (MODE == FFT_MODE_HS) {
      // weights: (A/c) 1/2 gz + A^2/2c^2 on F(Th psi), 1 on F(Th V psi), 1/2 (G+k)_i on
      // F(Th pi_i psi), plus (A/c) 1/2 on F(Th pi_z psi); S C = F(Th psi)
      const double gi = f == 2 ? gk[0] : f == 3 ? gk[1] : gk[2];
      const double w = f == 0 ? alpha_a * 0.5 * gk[2] + beta_a : f == 1 ? 1.0 : 0.5 * gi + (f == 4 ? 0.5 * alpha_a : 0.0);
      if (f == 0) a1 = val;
      a0 = f == 0 ? cscale(val, w) : cadd(a0, cscale(val, w));
    } else {  // TVPS: a0 T, a1 V, a2 P, a3 S
      if (f == 0) {
        a3 = val;
        a2 = cscale(val, 0.5 * gk[2]);
      } else if (f == 1) {
        a1 = val;
      } else {
        const double w = 0.5 * gk[f - 2];
        a0 = (f == 2) ? cscale(val, w) : cadd(a0, cscale(val, w));
        if (f == 4) a2 = cadd(a2, cscale(val, 0.5));
      }
    }
  }
  __device__ __forceinline__ void store(const FwdOut &fo, int gi, int col) const {
    const long long c = (long long)col;
    fo.o0[gi + c * fo.ld0] = a0;
    if constexpr (MODE != FFT_MODE_V) fo.o1[gi + c * fo.ld1] = a1;
    if constexpr (MODE == FFT_MODE_TVPS) {
      fo.o2[gi + c * fo.ld2] = a2;
      fo.o3[gi + c * fo.ld3] = a3;
    }
  }
};

// The apply's outputs at the sphere points from the five forward-transformed
// fields in sphere-table order (ys[f]: n_g x ncols, ld n_g, already scaled by
// 1/N): the sums of FwdAcc in registers, one store per output.  MODE_V: one field.
template <int MODE>
__global__ __launch_bounds__(256) void k_ap_combine(const FwdOut fo, const KSphere sp, const double2 *ys, int ncols,
                                                    double alpha_a, double beta_a) {
  constexpr int NF = MODE == FFT_MODE_V ? 1 : 5;
  const int ng = sp.n_g;
  const long long fs = (long long)ng * ncols;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < fs; e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e % ng), c = (int)(e / ng);
    const int gi = sp.pts_g[i];
    double gk[3] = {0.0, 0.0, 0.0};
    if constexpr (MODE != FFT_MODE_V)
#pragma unroll
      for (int d = 0; d < 3; ++d) gk[d] = sp.gk[3 * gi + d];
    double2 y[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) y[f] = ys[f * fs + e];
    FwdAcc<MODE> acc;
#pragma unroll
    for (int f = 0; f < NF; ++f) acc.add(f, y[f], gk, alpha_a, beta_a);
    acc.store(fo, gi, c);
  }
}

// Forward: per output field, the forward x transforms of the slab rows (only
// the box outputs kept, into the box columns; each pass's rows loaded during
// the previous pass), then the forward y transforms of the box columns in place
// (only |ky| <= by kept), then the field's term of each sphere point's outputs.
template <int N, int MODE>
__global__ __launch_bounds__(256, 2) void k_fwd_plane_reg(const Grid g, const FftKArgs ka, int ncols, double alpha_a,
                                                       double beta_a) {
  constexpr int F1 = 8, F2 = N / F1;
  using TT = Two<N, F1, F2>;
  constexpr int G = TT::G, LPW = TT::LPW, RP = rb_pitch(N), LS = TT::LS;
  constexpr int LO = zr_lo<N, F2>(), HI = zr_hi<N, F2>();
  constexpr int P2 = F2;  // exchange slots a P2 + d, a < F1, d < F2
  static_assert((F1 - 1) * P2 + F2 <= LS, "exchange scratch");
  constexpr int NF = MODE == FFT_MODE_V ? 1 : 5;
  constexpr int NP = (N + 4 * LPW - 1) / (4 * LPW);  // row passes per field
  extern __shared__ double2 sm_raw[];
  const int pz = blockIdx.x, col = blockIdx.y, kk = blockIdx.z;
  const int bx = g.bx, by = g.by, nbx = g.nbx;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane / G, r = lane - li * G;
  double2 *B = sm_raw;
  double *sd = reinterpret_cast<double *>(B + nbx * RP) + (wave * LPW + (li < LPW ? li : 0)) * LS;
  const KSphere &sp = ka.sph[kk];
  const FwdOut &fo = ka.out[kk];
  const int p0 = sp.plane_ptr[pz], p1 = sp.plane_ptr[pz + 1];
  constexpr long long plane_sz = (long long)N * N;
  const long long fstride = (long long)ncols * g.nbz * plane_sz;
  const double2 *src0 = ka.slab_in[kk] + ((long long)col * g.nbz + pz) * plane_sz;
  const double inv_n = 1.0 / ((double)N * N * g.n3);
  // this lane's twiddles exp(-2 pi i r j / N), j < F2
  double2 twt[F2];
#pragma unroll
  for (int j = 0; j < F2; ++j) twt[j] = g.tw1[(r * j) % N];
  // this thread's sphere points: G index, LDS slot of its box value (-1: none), (G+k)
  constexpr int PPT = MODE == FFT_MODE_TVPS ? 2 : PLANE_PPT;
  int pg[PPT], ps[PPT];
  double pk[PPT][3];
  FwdAcc<MODE> acc[PPT];
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int i = p0 + threadIdx.x + k * (int)blockDim.x;
    ps[k] = -1;
    pg[k] = 0;
    if (i < p1) {
      const int gi = sp.pts_g[i], xy = sp.pts_xy[i];
      const int y = xy / N, x = xy - y * N;
      pg[k] = gi;
      ps[k] = box_of(x, N, bx) * RP + (y <= by ? y : y - N) + by;
      if constexpr (MODE != FFT_MODE_V)
#pragma unroll
        for (int d = 0; d < 3; ++d) pk[k][d] = sp.gk[3 * gi + d];
    }
  }
  // rows of pass p of field f into u (lanes r < F1: x = r + F1 q)
  auto load_rows = [&](int f, int p, double2 (&u)[F2]) {
    const int y = wave * LPW + li + p * 4 * LPW;
    if (li < LPW && y < N && r < F1) {
      const double2 *src = src0 + f * fstride + (long long)y * N + r;
#pragma unroll
      for (int q = 0; q < F2; ++q) u[q] = src[F1 * q];
    }
  };
  double2 nxt[F2];
  load_rows(0, 0, nxt);
#pragma unroll 1
  for (int f = 0; f < NF; ++f) {
    // forward x transforms of the grid rows, box outputs into B[kx + bx][y]
#pragma unroll 1
    for (int p = 0; p < NP; ++p) {
      const int y = wave * LPW + li + p * 4 * LPW;
      const bool on = li < LPW && y < N;
      double2 u[F2], v[F1];
#pragma unroll
      for (int q = 0; q < F2; ++q) u[q] = nxt[q];
      if (p + 1 < NP) load_rows(f, p + 1, nxt);
      else if (f + 1 < NF) load_rows(f + 1, 0, nxt);
      if (on && r < F1) {
        dft_reg<F2, -1>(u);
        twiddle_tab<F2, -1>(u, twt);
      }
      xch_split<F2, F1>(sd, r, P2, on && r < F1, on && r < F2, u, v);
      if (on && r < F2) {
        dft_reg<F1, -1>(v);
#pragma unroll
        for (int c = 0; c < F1; ++c) {
          if (c >= LO && c <= HI) continue;  // |kx| > bx: never read
          const int m = F2 * c + r;
          if (m <= bx || m >= N - bx) B[(m <= bx ? m + bx : m - N + bx) * RP + y] = v[c];
        }
      }
      wave_fence();
    }
    __syncthreads();
    // forward y transforms of the box columns in place; |ky| <= by kept at B[b][ky + by]
    for (int b0 = wave * LPW; b0 < nbx; b0 += 4 * LPW) {
      const int b = b0 + li;
      const bool on = li < LPW && b < nbx;
      double2 *row = B + (on ? b : 0) * RP;
      if (on && r < F1) {
        double2 u[F2];
#pragma unroll
        for (int q = 0; q < F2; ++q) u[q] = row[r + F1 * q];
        dft_reg<F2, -1>(u);
        twiddle_tab<F2, -1>(u, twt);
        wave_fence();
#pragma unroll
        for (int d = 0; d < F2; ++d) row[r * F2 + d] = u[d];
      }
      wave_fence();
      double2 v[F1];
      if (on && r < F2) {
#pragma unroll
        for (int a = 0; a < F1; ++a) v[a] = row[a * F2 + r];
        dft_reg<F1, -1>(v);
      }
      wave_fence();
      if (on && r < F2) {
#pragma unroll
        for (int c = 0; c < F1; ++c) {
          if (c >= LO && c <= HI) continue;  // |ky| > by: never read
          const int m = F2 * c + r;
          if (m <= by || m >= N - by) row[m <= by ? m + by : m - N + by] = v[c];
        }
      }
      wave_fence();
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PPT; ++k)
      if (ps[k] >= 0) acc[k].add(f, cscale(B[ps[k]], inv_n), pk[k], alpha_a, beta_a);
    for (int i = p0 + threadIdx.x + PPT * (int)blockDim.x; i < p1; i += blockDim.x) {
      const int gi = sp.pts_g[i], xy = sp.pts_xy[i];
      const int y = xy / N, x = xy - y * N;
      const int ky = y <= by ? y : y - N;
      fwd_out_point(fo, sp, gi, col, f, MODE, cscale(B[box_of(x, N, bx) * RP + ky + by], inv_n), alpha_a, beta_a);
    }
    __syncthreads();  // the next field rewrites B
  }
#pragma unroll
  for (int k = 0; k < PPT; ++k)
    if (ps[k] >= 0) acc[k].store(fo, pg[k], col);
}

// ---------------------------------------------------------------------------
// Register-resident x/z transforms for N1' = N3' = 64 (box half-widths b <= 15,
// which the rebuild grid guarantees: 4 b + 1 <= 64).  One wavefront per
// (column, y') plane; each lane holds one whole 64-point transform in registers
// as 8 x 8: input n = 8 n1 + n2, output k = k1 + 8 k2, a first pass of length-8
// DFTs over n1, twiddles w^(n2 k1) (w = exp(DIR 2 pi i / 64)), a second pass over
// n2.  With |k| <= 15 the inputs with n1 in 2..5 are zero (the first pass drops
// them) and the outputs with k2 in 2..5 are never needed (never computed).
//   rows (x transforms): lane r < nbz takes box row r;
//   columns (z transforms): lane x takes grid column x.
// The plane's rows pass through the wave's own LDS slice R[nbz][65] between
// the phases (in-order LDS within a wave: wave fences, no block barrier).
// ---------------------------------------------------------------------------
constexpr double COS64[15] = {  // cos(2 pi j / 64), j = 1 .. 15
    0.9951847266721969,
    0.9807852804032304,
    0.9569403357322088,
    0.9238795325112867,
    0.881921264348355,
    0.8314696123025452,
    0.773010453362737,
    0.7071067811865476,
    0.6343932841636455,
    0.5555702330196023,
    0.4713967368259978,
    0.38268343236508984,
    0.29028467725446233,
    0.19509032201612833,
    0.09801714032956077};

// cos and sin of 2 pi j / 64 (compile-time j), exact at the multiples of pi/2
__host__ __device__ constexpr double cos64(int j) {
  j &= 63;
  const int q = j >> 4, r = j & 15;  // quadrant, offset
  const double c = r == 0 ? 1.0 : COS64[r - 1];   // cos of the offset
  const double s = r == 0 ? 0.0 : COS64[15 - r];  // its sin = cos(16 - r)
  return q == 0 ? c : q == 1 ? -s : q == 2 ? -c : s;
}
__host__ __device__ constexpr double sin64(int j) { return cos64(j - 16); }

// v * exp(DIR 2 pi i j / 64), j compile-time
template <int DIR, int J, class T>
__device__ __forceinline__ T tw64(T v) {
  using R = typename CT<T>::R;
  constexpr int j = J & 63;
  if constexpr (j == 0) return v;
  else if constexpr (j == 16) return mul_i<DIR>(v);
  else if constexpr (j == 32) return CT<T>::mk(-v.x, -v.y);
  else if constexpr (j == 48) return mul_i<-DIR>(v);
  else {
    constexpr double c = cos64(j), sn = DIR * sin64(j);
    return CT<T>::mk((R)c * v.x - (R)sn * v.y, (R)c * v.y + (R)sn * v.x);
  }
}

template <int DIR, int N2, int K1, class T>
__device__ __forceinline__ void tw_row(T (&y)[8][8]) {
  if constexpr (K1 < 8) {
    y[N2][K1] = tw64<DIR, N2 * K1>(y[N2][K1]);
    tw_row<DIR, N2, K1 + 1>(y);
  }
}
template <int DIR, int N2, class T>
__device__ __forceinline__ void tw_all(T (&y)[8][8]) {
  if constexpr (N2 < 8) {
    tw_row<DIR, N2, 1>(y);
    tw_all<DIR, N2 + 1>(y);
  }
}

// In-register 64-point DFT, natural order in and out: v_k = sum_n v_n w^(n k).
// INZ: inputs with n / 8 in 2..5 are zero; the outputs with k / 8 in 2..5 are
// left unset when the caller never reads them (dead code).
template <int DIR, bool INZ, class T>
__device__ __forceinline__ void fft64_reg(T (&v)[64]) {
  T y[8][8];  // y[n2][k1]
#pragma unroll
  for (int n2 = 0; n2 < 8; ++n2) {
    T u[8];
#pragma unroll
    for (int n1 = 0; n1 < 8; ++n1) u[n1] = v[8 * n1 + n2];
    if constexpr (INZ) dft8_z2345<DIR>(u);
    else dft8<DIR>(u);
#pragma unroll
    for (int k1 = 0; k1 < 8; ++k1) y[n2][k1] = u[k1];
    __builtin_amdgcn_sched_barrier(0);  // one group at a time (register pressure)
  }
  tw_all<DIR, 1>(y);
#pragma unroll
  for (int k1 = 0; k1 < 8; ++k1) {
    T u[8];
#pragma unroll
    for (int n2 = 0; n2 < 8; ++n2) u[n2] = y[n2][k1];
    dft8<DIR>(u);
#pragma unroll
    for (int k2 = 0; k2 < 8; ++k2) v[k1 + 8 * k2] = u[k2];
    __builtin_amdgcn_sched_barrier(0);
  }
}

// frequency index of position n of a 64-point transform, and whether n can be
// inside a box of half-width <= 15 (compile-time)
__host__ __device__ constexpr int freq64(int n) { return n <= 31 ? n : n - 64; }
__host__ __device__ constexpr bool box64(int n) { return (n >> 3) < 2 || (n >> 3) > 5; }

// LDS bytes of one plane's Theta V in k_rb_xzr (64 x 64 values at pitch 9 per x;
// the layout the x/z kernels read is [((y 8 + k2) 64 + x) 8 + k1], z = k1 + 8 k2)
template <class T>
__host__ __device__ constexpr size_t xzr_wbytes() {
  return ((size_t)8 * 64 * 9 * sizeof(typename CT<T>::R) + 15) / 16 * 16;
}

template <int NW, class T>
__global__ __launch_bounds__(NW * 64) void k_rb_xzr(const Grid g, const FftKArgs ka, int ncols,
                                                   const typename CT<T>::R *__restrict__ thp) {
  using RT = typename CT<T>::R;
  constexpr int RP = 65;  // LDS row pitch (odd)
  extern __shared__ double2 sm_raw[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = blockIdx.y, kk = blockIdx.z;
  const int y = blockIdx.x * NW + wave;
  const int n2 = g.n2, bx = g.bx, nbx = g.nbx, bz = g.bz, nbz = g.nbz;
  if (y >= n2) return;  // the whole wave; no block barrier in this kernel
  // per wave: Theta V of the plane, Wl[(k2 64 + x) 9 + k1] (pitch 9 per x: no
  // bank conflicts), then the rows R[nbz][RP]
  RT *Wl = reinterpret_cast<RT *>(reinterpret_cast<char *>(sm_raw) +
                                  (size_t)wave * (xzr_wbytes<T>() + (size_t)nbz * RP * sizeof(T)));
  T *R = reinterpret_cast<T *>(reinterpret_cast<char *>(Wl) + xzr_wbytes<T>());
  {  // Theta V of the plane: 4096 contiguous values, coalesced, into Wl
    const RT *src = thp + (long long)y * 4096;
#pragma unroll 16
    for (int it = 0; it < 64; ++it) {
      const int e = it * 64 + lane;
      Wl[(e >> 3) * 9 + (e & 7)] = src[e];
    }
  }
  const long long csz = (long long)nbz * n2 * nbx, rs = (long long)n2 * nbx;
  const T *in = reinterpret_cast<const T *>(ka.slab_in[kk]) + (long long)col * csz + (long long)y * nbx;
  T *out = reinterpret_cast<T *>(ka.slab_out[kk]) + (long long)col * csz + (long long)y * nbx;
  const T zero = CT<T>::mk(0, 0);
  T v[64];

  // phase 1: inverse x transform of box row `lane`
  if (lane < nbz) {
    const T *row = in + (long long)lane * rs;
#pragma unroll
    for (int n = 0; n < 64; ++n) {
      if (!box64(n)) {
        v[n] = zero;
      } else {
        const int kx = freq64(n);
        const int e = kx + bx < 0 ? 0 : (kx + bx > nbx - 1 ? nbx - 1 : kx + bx);
        const T t = row[e];
        v[n] = (kx >= -bx && kx <= bx) ? t : zero;
      }
    }
    fft64_reg<1, true>(v);
#pragma unroll
    for (int k = 0; k < 64; ++k) R[lane * RP + k] = v[k];
  }
  wave_fence();

  // phase 2: z column `lane`: inverse, times Theta V, forward (box outputs only).
  // The inverse's second pass for a fixed k1 yields z = k1 + 8 k2 (k2 = 0..7),
  // exactly the values the forward's first pass takes for n1 = k1, so the
  // product with Theta V runs group by group (eight of its values live at once).
  {
    const int x = lane;
#pragma unroll
    for (int n = 0; n < 64; ++n) {
      if (!box64(n)) {
        v[n] = zero;
      } else {
        const int kz = freq64(n);
        const int r = kz + bz < 0 ? 0 : (kz + bz > nbz - 1 ? nbz - 1 : kz + bz);
        const T t = R[r * RP + x];
        v[n] = (kz >= -bz && kz <= bz) ? t : zero;
      }
    }
    T yq[8][8];  // inverse first pass: yq[n2][k1]
#pragma unroll
    for (int n2 = 0; n2 < 8; ++n2) {
      T u[8];
#pragma unroll
      for (int n1 = 0; n1 < 8; ++n1) u[n1] = v[8 * n1 + n2];
      dft8_z2345<1>(u);
#pragma unroll
      for (int k1 = 0; k1 < 8; ++k1) yq[n2][k1] = u[k1];
      __builtin_amdgcn_sched_barrier(0);
    }
    tw_all<1, 1>(yq);
    T f[8][8];  // forward first pass output f[n1 = k1][m2]
#pragma unroll
    for (int k1 = 0; k1 < 8; ++k1) {
      RT wc[8];
#pragma unroll
      for (int k2 = 0; k2 < 8; ++k2) wc[k2] = Wl[(k2 * 64 + x) * 9 + k1];
      T t[8];
#pragma unroll
      for (int n2 = 0; n2 < 8; ++n2) t[n2] = yq[n2][k1];
      dft8<1>(t);  // t[k2]: the inverse at z = k1 + 8 k2
#pragma unroll
      for (int k2 = 0; k2 < 8; ++k2) t[k2] = cscale(t[k2], wc[k2]);
      dft8<-1>(t);  // over n2 = k2 for n1 = k1: t[m2]
#pragma unroll
      for (int m2 = 0; m2 < 8; ++m2) f[k1][m2] = t[m2];
      __builtin_amdgcn_sched_barrier(0);
    }
    tw_all<-1, 1>(f);  // w^(-n1 m2)
#pragma unroll
    for (int m2 = 0; m2 < 8; ++m2) {
      T u[8];
#pragma unroll
      for (int n1 = 0; n1 < 8; ++n1) u[n1] = f[n1][m2];
      dft8<-1>(u);  // u[m1]: output m = 8 m1 + m2
#pragma unroll
      for (int m1 = 0; m1 < 8; ++m1) {
        const int m = 8 * m1 + m2;
        if (!box64(m)) continue;
        const int kz = freq64(m);
        if (kz >= -bz && kz <= bz) R[(kz + bz) * RP + x] = u[m1];
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  wave_fence();

  // phase 3: forward x transform of box row `lane`, box columns out
  if (lane < nbz) {
#pragma unroll
    for (int n = 0; n < 64; ++n) v[n] = R[lane * RP + n];
    fft64_reg<-1, false>(v);
    T *orow = out + (long long)lane * rs;
#pragma unroll
    for (int m = 0; m < 64; ++m) {
      if (!box64(m)) continue;
      const int kx = freq64(m);
      if (kx >= -bx && kx <= bx) orow[kx + bx] = v[m];
    }
  }
}

// The same 8 x 8 transpose for complex64 lines, through a float2 scratch (the
// same slots: 8-byte accesses as in xch8_split).
__device__ __forceinline__ void xch8_split(float2 *sd, int r, const float2 (&in)[8], float2 (&out)[8]) {
#pragma unroll
  for (int k = 0; k < 8; ++k) sd[xslot<true>(r, k, 8)] = in[k];
  wave_fence();
#pragma unroll
  for (int q = 0; q < 8; ++q) out[q] = sd[xslot<true>(q, r, 8)];
  wave_fence();
}

// y transforms of the rebuild step for N2' = 64, nbx <= 32 and by <= 15: one
// block per (kz, column), one line per box x (4 waves x 8 lines x 8 lanes) from
// the first to the last x with a sphere point in the plane (the slab lines
// outside that range are never read out: about a fifth of them on a sphere).
// Each lane loads the values y = rx + 8 b of its line straight from the slab
// (eight 128-byte runs per load across a wave), runs the two-factor forward
// transform of k_rb_xz4's phase 3 with the exchange through a per-line scratch
// (lines 72 eight-byte slots apart; complex128 passes its real and imaginary
// parts in turn), and keeps the outputs with |ky| <= by in a box [x][ky] that
// takes the scratch's place; then the sphere read-out.  18 KB of LDS per block.
constexpr int Y64_LS = 72;
constexpr size_t y64_lds_bytes() { return (size_t)32 * Y64_LS * 8; }
template <class T>
__global__ __launch_bounds__(256) void k_rb_y64(const Grid g, const FftKArgs ka, int ncols) {
  constexpr int N = 64;
  using XT = typename std::conditional<sizeof(T) == 16, double, float2>::type;  // scratch slot type
  extern __shared__ double2 sm_raw[];
  XT *scr = reinterpret_cast<XT *>(sm_raw);
  T *box = reinterpret_cast<T *>(sm_raw);  // after the transforms: [x][ky + by], pitch nby
  const int pz = blockIdx.x, col = blockIdx.y, kk = blockIdx.z;
  const int nbx = g.nbx, bx = g.bx, by = g.by, nby = g.nby;
  const KSphere &sp = ka.sph[kk];
  const FwdOut &fo = ka.out[kk];
  const long long csz = (long long)g.nbz * N * nbx;
  const T *src = reinterpret_cast<const T *>(ka.slab_in[kk]) + (long long)col * csz + (long long)pz * N * nbx;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lx = lane >> 3, rx = lane & 7;
  // lines from the first box x with a sphere point in the plane to the last
  const int line = sp.plane_x[2 * pz] + wave * 8 + lx;
  const bool on = line < sp.plane_x[2 * pz + 1];
  // complex64: this thread's sphere points of the plane, read before the transforms
  constexpr int PP = sizeof(T) == 8 ? PLANE_PPT : 0;
  const int p0 = sp.plane_ptr[pz], p1 = sp.plane_ptr[pz + 1];
  int pxy[PP > 0 ? PP : 1];
#pragma unroll
  for (int k = 0; k < PP; ++k) {
    const int i = p0 + threadIdx.x + k * (int)blockDim.x;
    pxy[k] = i < p1 ? sp.pts_xy[i] : 0;
  }
  T v[8];
  if (on) {
    T twt[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) twt[j] = CT<T>::from(g.tw2[(rx * j) & 63]);
    T u[8];
#pragma unroll
    for (int b = 0; b < 8; ++b) u[b] = src[(rx + 8 * b) * nbx + line];
    dft8<-1>(u);
    twiddle_tab<8, -1>(u, twt);
    xch8_split(scr + line * Y64_LS, rx, u, v);
    dft8<-1>(v);
  }
  __syncthreads();  // every line has left the scratch
  if (on) {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      if (c >= 2 && c <= 5) continue;  // |ky| >= 16 > by
      const int m = 8 * c + rx;
      const int ky = m < 32 ? m : m - N;
      if (ky >= -by && ky <= by) box[line * nby + ky + by] = v[c];
    }
  }
  __syncthreads();
  const double inv_n = 1.0 / ((double)g.n1 * N * g.n3);
  const auto put = [&](int i, int xy) {
    const int yy = xy / g.d1, x = xy - yy * g.d1;
    const int ky = yy <= by ? yy : yy - g.d2;
    const double2 val = cscale(to_d2(box[box_of(x, g.d1, bx) * nby + ky + by]), inv_n);
    if (fo.o0f) fo.o0f[i + (long long)col * fo.ld0] = make_float2((float)val.x, (float)val.y);
    else fo.o0[i + (long long)col * fo.ld0] = val;
  };
#pragma unroll
  for (int k = 0; k < PP; ++k) {
    const int i = p0 + threadIdx.x + k * (int)blockDim.x;
    if (i < p1) put(i, pxy[k]);
  }
  for (int i = p0 + threadIdx.x + PP * (int)blockDim.x; i < p1; i += blockDim.x) put(i, sp.pts_xy[i]);
}

// y transforms of the rebuild step for N2' = 72 = 8 x 9 and nbx <= 35: one block
// per (kz, column), one line per box x (5 waves x 7 lines x 9 lanes) from the
// first to the last x with a sphere point in the plane.  Each lane
// a < 8 loads the values y = a + 8 b (b < 9) of its line from the slab, runs the
// forward two-factor transform of k_rb_xz4's phase 3 (length 9 over b, twiddles
// w^(a d) from a per-lane table, exchange through a per-line scratch, length 8
// over a) and keeps the outputs with |ky| <= by in a box [x][ky] that takes the
// scratch's place; then the sphere read-out.  PR (4 by + 1 <= 72): the outputs
// 9 c + d with c in 2..5 are never read and not computed.
constexpr int Y72_P = 9, Y72_LS = 73, Y72_LINES = 35;
inline size_t y72_lds_bytes(const Grid &g, size_t es) {
  const size_t scr = (size_t)Y72_LINES * Y72_LS * 8, box = (size_t)g.nbx * g.nby * es;
  return scr > box ? scr : box;
}
template <class T, bool PR>
__global__ __launch_bounds__(320) void k_rb_y72(const Grid g, const FftKArgs ka, int ncols) {
  constexpr int N = 72, F1 = 8, F2 = 9, LPW = 7;
  using XT = typename std::conditional<sizeof(T) == 16, double, float2>::type;  // scratch slot type
  extern __shared__ double2 sm_raw[];
  XT *scr = reinterpret_cast<XT *>(sm_raw);
  T *box = reinterpret_cast<T *>(sm_raw);  // after the transforms: [x][ky + by], pitch nby
  const int pz = blockIdx.x, col = blockIdx.y, kk = blockIdx.z;
  const int nbx = g.nbx, bx = g.bx, by = g.by, nby = g.nby;
  const KSphere &sp = ka.sph[kk];
  const FwdOut &fo = ka.out[kk];
  const long long csz = (long long)g.nbz * N * nbx;
  const T *src = reinterpret_cast<const T *>(ka.slab_in[kk]) + (long long)col * csz + (long long)pz * N * nbx;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lx = lane / F2, r = lane - lx * F2;
  // lines from the first box x with a sphere point in the plane to the last
  const int line = sp.plane_x[2 * pz] + wave * LPW + lx;
  const bool on = lx < LPW && line < sp.plane_x[2 * pz + 1];
  // complex64: this thread's sphere points of the plane, read before the
  // transforms (complex128: read at the read-out; the registers would cost a
  // wave per SIMD, measured 164 -> 182 us)
  constexpr int PP = sizeof(T) == 8 ? PLANE_PPT : 0;
  const int p0 = sp.plane_ptr[pz], p1 = sp.plane_ptr[pz + 1];
  int pxy[PP > 0 ? PP : 1];
#pragma unroll
  for (int k = 0; k < PP; ++k) {
    const int i = p0 + threadIdx.x + k * (int)blockDim.x;
    pxy[k] = i < p1 ? sp.pts_xy[i] : 0;
  }
  T v[F1];
  if (on) {
    XT *sl = scr + line * Y72_LS;
    T u[F2];
    if (r < F1) {
      T twt[F2];
#pragma unroll
      for (int j = 0; j < F2; ++j) twt[j] = CT<T>::from(g.tw2[(r * j) % N]);
#pragma unroll
      for (int b = 0; b < F2; ++b) u[b] = src[(r + F1 * b) * nbx + line];
      dft_reg<F2, -1>(u);
      twiddle_tab<F2, -1>(u, twt);
    }
    if constexpr (sizeof(T) == 16) {  // real parts, then imaginary parts (in-order LDS within a wave)
      if (r < F1)
#pragma unroll
        for (int d = 0; d < F2; ++d) sl[r * Y72_P + d] = u[d].x;
      wave_fence();
      if (r < F2)
#pragma unroll
        for (int a = 0; a < F1; ++a) v[a].x = sl[a * Y72_P + r];
      wave_fence();
      if (r < F1)
#pragma unroll
        for (int d = 0; d < F2; ++d) sl[r * Y72_P + d] = u[d].y;
      wave_fence();
      if (r < F2)
#pragma unroll
        for (int a = 0; a < F1; ++a) v[a].y = sl[a * Y72_P + r];
    } else {
      if (r < F1)
#pragma unroll
        for (int d = 0; d < F2; ++d) sl[r * Y72_P + d] = u[d];
      wave_fence();
      if (r < F2)
#pragma unroll
        for (int a = 0; a < F1; ++a) v[a] = sl[a * Y72_P + r];
    }
    if (r < F2) dft_reg<F1, -1>(v);
  }
  __syncthreads();  // every line has left the scratch
  if (on && r < F2) {
#pragma unroll
    for (int c = 0; c < F1; ++c) {
      if (PR && c >= 2 && c <= 5) continue;  // |ky| > 17 >= by
      const int m = F2 * c + r;
      const int ky = m < N / 2 ? m : m - N;
      if (ky >= -by && ky <= by) box[line * nby + ky + by] = v[c];
    }
  }
  __syncthreads();
  const double inv_n = 1.0 / ((double)g.n1 * N * g.n3);
  const auto put = [&](int i, int xy) {
    const int yy = xy / g.d1, x = xy - yy * g.d1;
    const int ky = yy <= by ? yy : yy - g.d2;
    const double2 val = cscale(to_d2(box[box_of(x, g.d1, bx) * nby + ky + by]), inv_n);
    if (fo.o0f) fo.o0f[i + (long long)col * fo.ld0] = make_float2((float)val.x, (float)val.y);
    else fo.o0[i + (long long)col * fo.ld0] = val;
  };
#pragma unroll
  for (int k = 0; k < PP; ++k) {
    const int i = p0 + threadIdx.x + k * (int)blockDim.x;
    if (i < p1) put(i, pxy[k]);
  }
  for (int i = p0 + threadIdx.x + PP * (int)blockDim.x; i < p1; i += blockDim.x) put(i, sp.pts_xy[i]);
}

// One axis pass of the W synthesis with the axis matrix given by its Dirichlet
// table: M[j'][j] = tab[(c1 j' - c2 j) mod L] (c1 = N/g, c2 = N'/g, L = N N'/g,
// g = gcd(N, N')), so that the block stages L values instead of N' N.
//   out(o, j', i) = sum_j M[j'][j] f(o, j, i),  f(o, j, i) = in[(o N + j) I + i]
//   (times th[...] when th is given), o < O, j' < Np, i < I.
// A block takes TP positions p = o I + i (i fastest) and all j'.  perm_n1 > 0:
// the z pass into the k_rb_xz4 order (O = 1, i = y' N1' + x').
// LDS: table [L], tile [N][TP+1].
// TO: output type (float for the FP32 residual); sub != NULL (z pass): the
// output is acc - sub[same index] (W(t) - W_ref).
template <int TP, bool TH, class TO>
__global__ __launch_bounds__(256) void k_syn_pass(const double *__restrict__ in, const double *__restrict__ th,
                                                  const int *step, long long stride, TO *__restrict__ out,
                                                  const double *__restrict__ sub,
                                                  const double *__restrict__ tab, int L, int c1, int c2, int O,
                                                  int N, int I, int Np, int perm_n1, int perm_z1, int perm_z2) {
  extern __shared__ double sd[];
  double *tb = sd;
  double *T = sd + L;
  const int P = O * I;
  const int p0 = blockIdx.x * TP;
  const int np = (P - p0) < TP ? (P - p0) : TP;
  if (step) in += (long long)(*step) * stride;
  stage8<double>(
      L, [&](int e) { return tab[e]; }, [&](int e, double x) { tb[e] = x; });
  if (I == 1) {  // rows o = p, contiguous in j
    stage8<double>(
        np * N,
        [&](int e) {
          const long long src = (long long)p0 * N + e;
          if constexpr (TH) return th[src] * in[src];
          else return in[src];
        },
        [&](int e, double x) { T[(e % N) * (TP + 1) + e / N] = x; });
  } else {  // positions contiguous in i (at most one row boundary: TP <= I)
    const int o0 = p0 / I, i0 = p0 - o0 * I;
    stage8<double>(
        N * TP,
        [&](int e) {
          const int j = e / TP, pl = e % TP;
          int i = i0 + (pl < np ? pl : np - 1), o = o0;
          if (i >= I) {
            i -= I;
            ++o;
          }
          const long long src = ((long long)o * N + j) * I + i;
          if constexpr (TH) return th[src] * in[src];
          else return in[src];
        },
        [&](int e, double x) { T[(e / TP) * (TP + 1) + e % TP] = x; });
  }
  __syncthreads();
  // 2 x 2 output tiles (j', position); the table index of row j' at j is
  // (c1 j' - c2 j) mod L, stepped by -c2 (mod L) along j
  const int tn = (np + 1) / 2, tiles = ((Np + 1) / 2) * tn;
  for (int tile = threadIdx.x; tile < tiles; tile += blockDim.x) {
    const int i0 = (tile / tn) * 2, q0 = (tile % tn) * 2;
    const int ra = i0, rb = (i0 + 1 < Np) ? i0 + 1 : Np - 1;
    const int qa = q0, qb = (q0 + 1 < np) ? q0 + 1 : np - 1;
    int xa = (int)(((long long)c1 * ra) % L), xb = (int)(((long long)c1 * rb) % L);
    double s00 = 0.0, s01 = 0.0, s10 = 0.0, s11 = 0.0;
#pragma unroll 8
    for (int j = 0; j < N; ++j) {
      const double ma = tb[xa], mb = tb[xb];
      const double ta = T[j * (TP + 1) + qa], tq = T[j * (TP + 1) + qb];
      s00 = fma(ma, ta, s00);
      s01 = fma(ma, tq, s01);
      s10 = fma(mb, ta, s10);
      s11 = fma(mb, tq, s11);
      xa -= c2;
      xa += xa < 0 ? L : 0;
      xb -= c2;
      xb += xb < 0 ? L : 0;
    }
    const double acc[2][2] = {{s00, s01}, {s10, s11}};
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int jp = i0 + r, q = q0 + c;
        if (jp >= Np || q >= np) continue;
        const int p = p0 + q, o = p / I, i = p - o * I;
        if (perm_n1 > 0) {
          const int y = i / perm_n1, x = i - y * perm_n1;
          const long long oi = (((long long)y * perm_z2 + jp / perm_z1) * perm_n1 + x) * perm_z1 + jp % perm_z1;
          out[oi] = (TO)(sub ? acc[r][c] - sub[oi] : acc[r][c]);
        } else {
          out[((long long)o * Np + jp) * I + i] = (TO)acc[r][c];
        }
      }
  }
}


// The same axis pass on the matrix cores (v_mfma_f64_16x16x4f64), for N a
// multiple of 4 (KS = N / 4 steps of K = 4).  The axis matrix comes as MFMA
// fragments mf[(s RB + a) 64 + lane] = M[16 a + lane % 16][4 s + lane / 16]
// (zero outside Np x N, RB = ceil(Np / 16)).  A wave computes one 16 x 16
// output block:
//  ROWS (I == 1, the positions are the rows o, contiguous in j): a block of
//    RB waves takes 16 rows, staged through LDS; the data rows are the A
//    operand and M^T the B operand, D[p][j'] = sum_j F[p][j] M[j'][j], so the 16
//    lanes of an output register write 16 consecutive j';
//  otherwise (a block of 16 consecutive positions p = o I + i, which may cross
//    from one o to the next when I is not a multiple of 16): M is the A operand
//    and the data the B operand, D[j'][p] = sum_j M[j'][j] F[j][p], each lane
//    reading and writing at its own position.
// Output element of accumulator register r: row 4 r + lane / 16, column lane % 16.
template <int KS, bool ROWS, bool TH, class TO>
__global__ __launch_bounds__(512) void k_syn_mfma(const double *__restrict__ in, const double *__restrict__ th,
                                                  const int *step, long long stride, TO *__restrict__ out,
                                                  const double *__restrict__ sub, const double *__restrict__ mf,
                                                  int RB, int O, int N, int I, int Np, int perm_n1, int perm_z1,
                                                  int perm_z2) {
  typedef double d4 __attribute__((ext_vector_type(4)));
  constexpr int RP = 4 * KS + 1;  // LDS row pitch of the ROWS tile (odd: no bank conflicts)
  __shared__ double tile[ROWS ? 16 * RP : 1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long P = (long long)O * I;
  const int lr = lane & 15, lk = lane >> 4;
  if (step) in += (long long)(*step) * stride;
  double fa[KS], fb[KS];
  int a;
  long long p0;
  if constexpr (ROWS) {
    // a block is 16 consecutive rows (contiguous in memory), staged once through
    // LDS with coalesced loads; its RB waves are the 16-column blocks of j'
    p0 = (long long)blockIdx.x * 16;
    a = wave;
    const int nr = P - p0 < 16 ? (int)(P - p0) : 16;
    const double *src = in + p0 * N;
    const double *ths = TH ? th + p0 * N : nullptr;
    stage8<double>(
        nr * N,
        [&](int e) {
          if constexpr (TH) return ths[e] * src[e];
          else return src[e];
        },
        [&](int e, double x) { tile[(e / N) * RP + e % N] = x; });
    __syncthreads();
    if (a >= RB) return;
    const int rr = lr < nr ? lr : nr - 1;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      fa[s] = tile[rr * RP + 4 * s + lk];
      fb[s] = mf[(s * RB + a) * 64 + lane];
    }
  } else {
    const long long task = (long long)blockIdx.x * (blockDim.x >> 6) + wave;
    const long long ntile = (P + 15) / 16;
    if (task >= ntile * RB) return;  // the whole wave (task is uniform across it)
    a = (int)(task % RB);
    p0 = (task / RB) * 16;
    const long long pl = p0 + lr < P ? p0 + lr : P - 1;  // this lane's position (clamped)
    const long long o = pl / I;
    const long long i = pl - o * I;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const long long src = (o * N + 4 * s + lk) * I + i;
      if constexpr (TH) fb[s] = th[src] * in[src];
      else fb[s] = in[src];
      fa[s] = mf[(s * RB + a) * 64 + lane];
    }
  }
  d4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s = 0; s < KS; s += 2) {
    acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[s], fb[s], acc0, 0, 0, 0);
    if (s + 1 < KS) acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[s + 1], fb[s + 1], acc1, 0, 0, 0);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const double v = acc0[r] + acc1[r];
    if constexpr (ROWS) {
      const long long p = p0 + 4 * r + lk;
      const int jp = 16 * a + lr;
      if (p < P && jp < Np) out[p * Np + jp] = (TO)v;
    } else {
      const int jp = 16 * a + 4 * r + lk;
      const long long p = p0 + lr;
      const long long o = p / I;
      const long long i = p - o * I;
      if (jp >= Np || p >= P) continue;
      if (perm_n1 > 0) {
        const long long y = i / perm_n1, x = i - y * perm_n1;
        const long long oi = ((y * perm_z2 + jp / perm_z1) * perm_n1 + x) * perm_z1 + jp % perm_z1;
        out[oi] = (TO)(sub ? v - sub[oi] : v);
      } else {
        out[(o * Np + jp) * I + i] = (TO)v;
      }
    }
  }
}

// Theta V in the order k_rb_xz4 reads it: out[((y Z2 + k2) N1 + x) Z1 + k1] for
// the grid point (z = k1 + Z1 k2, y, x); z1 == 0: the grid order itself.
// vref != NULL: Theta (v - vref) (the residual, in TO = float).
template <class TO>
__global__ void k_rb_thv(TO *__restrict__ out, const double *__restrict__ th, const double *__restrict__ v,
                         const double *__restrict__ vref, const int *step, long long stride, int n1, int n2, int n3,
                         int z1, int z2) {
  const long long ng = (long long)n1 * n2 * n3;
  if (step) v += (long long)(*step) * stride;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < ng; i += (long long)gridDim.x * blockDim.x) {
    if (z1 == 0) {
      out[i] = (TO)(th[i] * (vref ? v[i] - vref[i] : v[i]));
      continue;
    }
    const int x = (int)(i % n1);
    const long long t = i / n1;
    const int y = (int)(t % n2), z = (int)(t / n2);
    const int k1 = z % z1, k2 = z / z1;
    out[(((long long)y * z2 + k2) * n1 + x) * z1 + k1] = (TO)(th[i] * (vref ? v[i] - vref[i] : v[i]));
  }
}

// ---------------------------------------------------------------------------
// Launch configuration
// ---------------------------------------------------------------------------
// rows per chunk of the plane passes: every wavefront transforms its full share of lines
int plane_ch(const Grid &g) {
  const int ch = (FFT_NT / 64) * lines_per_wave(g.p1);
  return ch < g.n2 ? ch : g.n2;
}

size_t plane_lds(const Grid &g) {
  return ((size_t)g.nbx * (g.n2 + 1) + (size_t)plane_ch(g) * (g.n1 + 1) + g.n1 + g.n2) * sizeof(double2);
}

int line_tile(const Grid &g, bool vmode) {
  const long long plane_sz = (long long)g.n1 * g.n2;
  const int nbuf = vmode ? 1 : 2;
  const size_t budget = vmode ? 40 * 1024 : 52 * 1024;
  int t = 64;
  while (t > 8 && (size_t)(nbuf * g.n3 * (t + 1) + g.n3) * sizeof(double2) > budget) t /= 2;
  while (t > 8 && t / 2 >= plane_sz) t /= 2;
  return t;
}

size_t line_lds(const Grid &g, int t, bool vmode) {
  return (size_t)((vmode ? 1 : 2) * g.n3 * (t + 1) + g.n3) * sizeof(double2);
}

size_t rb_cache_lds(const Grid &g, size_t es = sizeof(double2)) { return ((size_t)g.nbx * (g.n2 + 1) + g.n2) * es; }

// x columns per z chunk of k_rb_xz: the fewest equal chunks that keep the block
// within 80 KB of LDS (two blocks per CU), else within the 160 KB of one CU
int rb_xc(const Grid &g) {
  const size_t fixed = ((size_t)g.nbz * (g.n1 + 1) + g.n1 + g.n3) * sizeof(double2);
  for (size_t budget : {(size_t)80 * 1024, (size_t)160 * 1024})
    for (int nch = 1; nch <= g.n1; ++nch) {
      const int xc = (g.n1 + nch - 1) / nch;
      if (fixed + (size_t)g.n3 * (xc + 1) * sizeof(double2) <= budget) return xc;
    }
  return 1;
}

size_t rb_xz_lds(const Grid &g) {
  return ((size_t)g.nbz * (g.n1 + 1) + (size_t)g.n3 * (rb_xc(g) + 1) + g.n1 + g.n3) * sizeof(double2);
}

// Launch shapes of k_rb_xz4 (waves per block, z columns per wave), the
// candidates of the tuner: 0 = (4, LZ), 1 = (2, LZ), 2 = (4, LZ / 2), LZ as rb_lz.
constexpr int RB_VARIANTS = 3;  // launch shapes of k_rb_xz4; shape RB_VARIANTS is k_rb_xzr
// planes (waves) per block of k_rb_xzr: its LDS (Theta V and rows per plane) within 160 KB.
// Only the complex64 instance is launched: 64 complex128 values per lane would
// not fit the 256 architectural VGPRs.
template <class T>
constexpr int xzr_nw() { return sizeof(T) == 16 ? 2 : 4; }
constexpr int rb_nw_of(int v) { return v == 1 ? 2 : 4; }
template <int NZ, int Z1>
constexpr int rb_lz_of(int v) {
  return v == 2 ? (rb_lz(Two<NZ, Z1, NZ / Z1>::LPW) / 2 > 0 ? rb_lz(Two<NZ, Z1, NZ / Z1>::LPW) / 2 : 1)
                : rb_lz(Two<NZ, Z1, NZ / Z1>::LPW);
}

// the three launch shapes of the x/z kernel for x length NX = X1 (NX / X1) and z
// length NZ = Z1 (NZ / Z1)
template <int NX, int X1, int NZ, int Z1, class T, bool PR, class F>
void reg_xz4(F &&f) {
  f((const void *)k_rb_xz4<NX, X1, NX / X1, NZ, Z1, NZ / Z1, rb_nw_of(0), rb_lz_of<NZ, Z1>(0), T, PR>);
  f((const void *)k_rb_xz4<NX, X1, NX / X1, NZ, Z1, NZ / Z1, rb_nw_of(1), rb_lz_of<NZ, Z1>(1), T, PR>);
  f((const void *)k_rb_xz4<NX, X1, NX / X1, NZ, Z1, NZ / Z1, rb_nw_of(2), rb_lz_of<NZ, Z1>(2), T, PR>);
}
// the lengths whose lines are pruned when the box fits the exact-grid bound
template <int NX, int NZ>
constexpr bool xz4_prunable() { return (NX == 72 && (NZ == 72 || NZ == 108)); }

template <int NX, int X1, int NZ, int Z1, class T, bool PR>
void launch_xz4_pr(const Grid &g, const FftKArgs &ka, int nk, int ncols, const void *thv, hipStream_t s, int v) {
  const auto *th = static_cast<const typename CT<T>::R *>(thv);
  const dim3 grid(ncols, g.n2, nk);
#define LTD_V(V)                                                                                       \
  do {                                                                                                 \
    constexpr int NW = rb_nw_of(V), LZ = rb_lz_of<NZ, Z1>(V);                                          \
    const size_t lds = xz4_lds<NX, X1, NZ, Z1, T>(g.nbz, NW, LZ);                                      \
    hipLaunchKernelGGL((k_rb_xz4<NX, X1, NX / X1, NZ, Z1, NZ / Z1, NW, LZ, T, PR>), grid, dim3(NW * 64), \
                       lds, s, g, ka, ncols, th);                                                      \
  } while (0)
  if (v == 1) LTD_V(1);
  else if (v == 2) LTD_V(2);
  else LTD_V(0);
#undef LTD_V
}

template <int NX, int X1, int NZ, int Z1, class T>
void launch_xz4(const Grid &g, const FftKArgs &ka, int nk, int ncols, const void *thv, hipStream_t s, int v) {
  if constexpr (xz4_prunable<NX, NZ>()) {
    if (4 * g.bx + 1 <= NX && 4 * g.bz + 1 <= NZ) {
      launch_xz4_pr<NX, X1, NZ, Z1, T, true>(g, ka, nk, ncols, thv, s, v);
      return;
    }
  }
  launch_xz4_pr<NX, X1, NZ, Z1, T, false>(g, ka, nk, ncols, thv, s, v);
}

template <class F>
void each_plane_kernel(F &&f) {
  f((const void *)k_rb_xz<0, 0>);
#define LTD_RB(a, c)                            \
  f((const void *)k_rb_cache<a, double2>);      \
  f((const void *)k_rb_cache<a, float2>);       \
  f((const void *)k_rb_y<a, double2>);          \
  f((const void *)k_rb_y<a, float2>);           \
  f((const void *)k_rb_xz<a, c>);
  LTD_RB(0, 0) LTD_RB(16, 16) LTD_RB(64, 64) LTD_RB(72, 72) LTD_RB(96, 160)
#undef LTD_RB
  reg_xz4<72, 8, 72, 8, double2, false>(f);
  reg_xz4<64, 8, 64, 8, double2, false>(f);
  reg_xz4<16, 4, 16, 4, double2, false>(f);
  reg_xz4<72, 8, 108, 12, double2, false>(f);
  reg_xz4<72, 8, 72, 8, float2, false>(f);
  reg_xz4<64, 8, 64, 8, float2, false>(f);
  reg_xz4<16, 4, 16, 4, float2, false>(f);
  reg_xz4<72, 8, 108, 12, float2, false>(f);
  reg_xz4<72, 8, 72, 8, double2, true>(f);
  reg_xz4<72, 8, 108, 12, double2, true>(f);
  reg_xz4<72, 8, 72, 8, float2, true>(f);
  reg_xz4<72, 8, 108, 12, float2, true>(f);
  f((const void *)k_rb_xzr<xzr_nw<float2>(), float2>);
  f((const void *)k_inv_plane<0, 0>);
  f((const void *)k_fwd_plane<0, 0>);
  f((const void *)k_inv_plane_reg<72>);
  f((const void *)k_inv_plane_reg<64>);
#define LTD_FR(a)                                          \
  f((const void *)k_fwd_plane_reg<a, FFT_MODE_V>);         \
  f((const void *)k_fwd_plane_reg<a, FFT_MODE_HS>);        \
  f((const void *)k_fwd_plane_reg<a, FFT_MODE_TVPS>);
  LTD_FR(72) LTD_FR(64)
#undef LTD_FR
#define LTD_PL(a, b)                            \
  f((const void *)k_inv_plane<a, b>);           \
  f((const void *)k_fwd_plane<a, b>);
  LTD_PL(16, 16) LTD_PL(64, 64) LTD_PL(72, 72) LTD_PL(96, 96)
#undef LTD_PL
#define LTD_LK(a)                               \
  f((const void *)k_lines<a, true>);            \
  f((const void *)k_lines<a, false>);
  LTD_LK(0) LTD_LK(16) LTD_LK(64) LTD_LK(72) LTD_LK(108) LTD_LK(160)
#undef LTD_LK
}

bool attrs_set = false;
void set_attrs() {
  if (attrs_set) return;
  each_plane_kernel([](const void *k) {
    (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  });
  attrs_set = true;
}

}  // namespace

bool fft_plan_length(int L, FftPlan *p) {
  if (L < 2 || L > FFT_MAXLEN) return false;
  const Radices f = factor_len(L);
  int prod = 1;
  for (int s = 0; s < f.n; ++s) prod *= f.r[s];
  if (prod != L) return false;
  p->L = L;
  p->nst = f.n;
  for (int s = 0; s < f.n; ++s) p->radix[s] = f.r[s];
  // one wavefront must hold at least one line in every pass
  for (int s = 0; s < p->nst; ++s)
    if (L / p->radix[s] > 64 * tpl_of(p->radix[s])) return false;
  return true;
}

void fft_init_attrs() { set_attrs(); }

size_t fft_rb_slab_values(const Grid &g) { return (size_t)g.nbz * g.n2 * g.nbx; }

// Two-factor splits N = F1 F2 of the x and z lengths with a register path (F1, or 0 if none).
int rb_split(int n) { return n == 72 ? 8 : n == 64 ? 8 : n == 16 ? 4 : n == 108 ? 12 : 0; }
// (x, z) length pairs of the register x/z kernel
bool rb_pair(int nx, int nz) {
  return (nx == nz && (nx == 16 || nx == 64 || nx == 72)) || (nx == 72 && nz == 108);
}
// the register x/z kernel; on 64-point axes it drops the inputs and outputs with
// |frequency| >= 16, so the box there must have b <= 15 (which 64 >= 4 b + 1 gives)
bool rb_fast(const Grid &g) {
  const auto ok = [](int n, int b) { return rb_split(n) > 0 && (n != 64 || b <= 15); };
  return rb_pair(g.n1, g.n3) && ok(g.n1, g.bx) && ok(g.n3, g.bz);
}


bool fft_rb_fast(const Grid &g) { return rb_fast(g); }

int fft_rb_length(int n, int b) {
  for (int c : {16, 64, 72, 108})
    if (c >= 4 * b + 1 && c <= n) return c;
  return n;
}

int fft_rb_table_len(int n, int np) { return n / std::gcd(n, np) * np; }

int fft_rb_frag_len(int n, int np) { return ((np + 15) / 16) * ((n + 3) / 4) * 64; }

void fft_rb_frag(int n, int np, const double *tab, double *mf) {
  const int g = std::gcd(n, np), L = n / g * np, c1 = n / g, c2 = np / g;
  const int rb = (np + 15) / 16, ks = (n + 3) / 4;
  for (int s = 0; s < ks; ++s)
    for (int a = 0; a < rb; ++a)
      for (int l = 0; l < 64; ++l) {
        const int jp = 16 * a + l % 16, j = 4 * s + l / 16;
        double v = 0.0;
        if (jp < np && j < n) {
          long long m = ((long long)c1 * jp - (long long)c2 * j) % L;
          if (m < 0) m += L;
          v = tab[m];
        }
        mf[((size_t)s * rb + a) * 64 + l] = v;
      }
}

namespace {
// MFMA pass for N in {16, 64, 72, 96, 160} (ROWS: at most eight 16-row blocks of
// j', one wave each); false when the shape has no instantiation
template <bool ROWS, bool TH, class TO>
bool syn_mfma(int N, dim3 grid, hipStream_t s, const double *in, const double *th, const int *step, long long stride,
              TO *out, const double *sub, const double *mf, int RB, int O, int I, int Np, int pn1, int z1, int z2) {
  if (ROWS && (I != 1 || RB > 8)) return false;
  if (ROWS) grid = dim3((unsigned)(((long long)O + 15) / 16));
  const dim3 block(ROWS ? 64 * RB : 256);
#define LTD_SM(KS) \
  hipLaunchKernelGGL((k_syn_mfma<KS, ROWS, TH, TO>), grid, block, 0, s, in, th, step, stride, out, sub, mf, RB, O, N, \
                     I, Np, pn1, z1, z2)
  switch (N) {
    case 16: LTD_SM(4); return true;
    case 64: LTD_SM(16); return true;
    case 72: LTD_SM(18); return true;
    case 96: LTD_SM(24); return true;
    case 160: LTD_SM(40); return true;
    default: return false;
  }
#undef LTD_SM
}
}  // namespace

hipError_t fft_rb_synth(const Grid &gr, int n1, int n2, int n3, const double *th, const double *v,
                        const int *step, long long stride, const double *tab1, const double *tab2,
                        const double *tab3, const double *mf1, const double *mf2, const double *mf3, double *t1,
                        double *t2, void *out, const double *sub, bool fp32, hipStream_t s, bool plain) {
  static bool attr = false;
  if (!attr) {
    for (const void *k : {(const void *)k_syn_pass<32, true, double>, (const void *)k_syn_pass<16, false, double>,
                          (const void *)k_syn_pass<16, false, float>})
      (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    attr = true;
  }
  const int z1 = rb_split(gr.n3), z2 = gr.n3 / z1;
  const auto pass = [&](auto kern, int tp, const double *in, const double *thp, const int *st, auto *o,
                        const double *sb, const double *tab, int n, int np, int O, int I, int pn1) {
    const int g = std::gcd(n, np), L = n / g * np;
    const size_t lds = ((size_t)L + (size_t)n * (tp + 1)) * sizeof(double);
    const int P = O * I;
    hipLaunchKernelGGL(kern, dim3((P + tp - 1) / tp), dim3(256), lds, s, in, thp, st, stride, o, sb, tab, L, n / g,
                       np / g, O, n, I, np, pn1, z1, z2);
  };
  const auto grid_of = [](int np, long long P) {
    const long long tasks = ((np + 15) / 16) * ((P + 15) / 16);
    return dim3((unsigned)((tasks + 3) / 4));
  };
  const auto rb = [](int np) { return (np + 15) / 16; };
  // x: [n3 n2][n1] -> [n3 n2][n1']  (Theta V formed on the fly)
  if (!syn_mfma<true, true, double>(n1, grid_of(gr.n1, (long long)n3 * n2), s, v, th, step, stride, t1, nullptr, mf1,
                                    rb(gr.n1), n3 * n2, 1, gr.n1, 0, z1, z2))
    pass(k_syn_pass<32, true, double>, 32, v, th, step, t1, nullptr, tab1, n1, gr.n1, n3 * n2, 1, 0);
  // y: [n3][n2][n1'] -> [n3][n2'][n1']  (16 <= n1': one row boundary at most per block)
  if (!syn_mfma<false, false, double>(n2, grid_of(gr.n2, (long long)n3 * gr.n1), s, t1, nullptr, nullptr, 0, t2,
                                      nullptr, mf2, rb(gr.n2), n3, gr.n1, gr.n2, 0, z1, z2))
    pass(k_syn_pass<16, false, double>, 16, t1, nullptr, nullptr, t2, nullptr, tab2, n2, gr.n2, n3, gr.n1, 0);
  // z: [n3][n2' n1'] -> the k_rb_xz4 order (minus sub, in FP32 for the residual)
  const long long pz = (long long)gr.n2 * gr.n1;
  const int pn = plain ? 0 : gr.n1;  // 0: grid order
  if (fp32) {
    if (!syn_mfma<false, false, float>(n3, grid_of(gr.n3, pz), s, t2, nullptr, nullptr, 0, static_cast<float *>(out),
                                       sub, mf3, rb(gr.n3), 1, (int)pz, gr.n3, pn, z1, z2))
      pass(k_syn_pass<16, false, float>, 16, t2, nullptr, nullptr, static_cast<float *>(out), sub, tab3, n3, gr.n3, 1,
           gr.n2 * gr.n1, pn);
  } else {
    if (!syn_mfma<false, false, double>(n3, grid_of(gr.n3, pz), s, t2, nullptr, nullptr, 0,
                                        static_cast<double *>(out), sub, mf3, rb(gr.n3), 1, (int)pz, gr.n3, pn, z1,
                                        z2))
      pass(k_syn_pass<16, false, double>, 16, t2, nullptr, nullptr, static_cast<double *>(out), sub, tab3, n3, gr.n3,
           1, gr.n2 * gr.n1, pn);
  }
  return hipGetLastError();
}

hipError_t fft_rb_thv(const Grid &g, const double *th, const double *v, const int *step, long long stride,
                      void *out, const double *vref, bool fp32, hipStream_t s) {
  const int z1 = rb_fast(g) ? rb_split(g.n3) : 0, z2 = z1 ? g.n3 / z1 : 0;
  const long long ng = (long long)g.n1 * g.n2 * g.n3;
  const int blocks = (int)std::min<long long>((ng + 255) / 256, 4096);
  if (fp32)
    hipLaunchKernelGGL(k_rb_thv<float>, dim3(blocks), dim3(256), 0, s, static_cast<float *>(out), th, v, vref, step,
                       stride, g.n1, g.n2, g.n3, z1, z2);
  else
    hipLaunchKernelGGL(k_rb_thv<double>, dim3(blocks), dim3(256), 0, s, static_cast<double *>(out), th, v, vref, step,
                       stride, g.n1, g.n2, g.n3, z1, z2);
  return hipGetLastError();
}

hipError_t fft_rb_cache(const Grid &g, const FftKArgs &ka, int nk, int ncols, hipStream_t s, bool fp32) {
  set_attrs();
  const dim3 grid(g.nbz, ncols, nk), block(FFT_NT);
  const size_t lds = rb_cache_lds(g, fp32 ? sizeof(float2) : sizeof(double2));
#define LTD_RC(a)                                                                    \
  do {                                                                               \
    if (fp32) hipLaunchKernelGGL((k_rb_cache<a, float2>), grid, block, lds, s, g, ka, ncols); \
    else hipLaunchKernelGGL((k_rb_cache<a, double2>), grid, block, lds, s, g, ka, ncols);     \
  } while (0)
  if (g.n2 == 16) LTD_RC(16);
  else if (g.n2 == 64) LTD_RC(64);
  else if (g.n2 == 72) LTD_RC(72);
  else if (g.n2 == 96) LTD_RC(96);
  else LTD_RC(0);
#undef LTD_RC
  return hipGetLastError();
}

int fft_rb_variants(const Grid &g, bool fp32) {
  return (fp32 && g.n1 == 64 && g.n3 == 64 && g.bx <= 15 && g.bz <= 15) ? RB_VARIANTS + 1 : RB_VARIANTS;
}

namespace {
template <class T>
void launch_xzr(const Grid &g, const FftKArgs &ka, int nk, int ncols, const void *thv, hipStream_t s) {
  constexpr int NW = xzr_nw<T>();
  const dim3 grid((g.n2 + NW - 1) / NW, ncols, nk), block(64 * NW);
  const size_t lds = (size_t)NW * (xzr_wbytes<T>() + (size_t)g.nbz * 65 * sizeof(T));
  hipLaunchKernelGGL((k_rb_xzr<NW, T>), grid, block, lds, s, g, ka, ncols,
                     static_cast<const typename CT<T>::R *>(thv));
}
}  // namespace

hipError_t fft_rb_step(const Grid &g, const FftKArgs &ka, int nk, int ncols, const void *thv, hipStream_t s,
                       int part, bool fp32, int variant) {
  set_attrs();
  const dim3 block(FFT_NT);
  if (variant < 0 || variant >= fft_rb_variants(g, fp32)) return hipErrorInvalidValue;
  if (part == 0 && variant == RB_VARIANTS) {  // register-resident: complex64 on 64-point grids
    launch_xzr<float2>(g, ka, nk, ncols, thv, s);
  } else if (part == 0 && rb_fast(g)) {
#define LTD_XZ4P(nx, x1, nz, z1)                                                    \
  do {                                                                              \
    if (fp32) launch_xz4<nx, x1, nz, z1, float2>(g, ka, nk, ncols, thv, s, variant);  \
    else launch_xz4<nx, x1, nz, z1, double2>(g, ka, nk, ncols, thv, s, variant);      \
  } while (0)
    if (g.n1 == 72 && g.n3 == 72) LTD_XZ4P(72, 8, 72, 8);
    else if (g.n1 == 64 && g.n3 == 64) LTD_XZ4P(64, 8, 64, 8);
    else if (g.n1 == 16 && g.n3 == 16) LTD_XZ4P(16, 4, 16, 4);
    else if (g.n1 == 72 && g.n3 == 108) LTD_XZ4P(72, 8, 108, 12);
    else return hipErrorInvalidValue;
#undef LTD_XZ4P
  } else if (part == 0) {
    if (fp32) return hipErrorInvalidValue;  // the FP32 residual needs the register path
    const dim3 grid(ncols, g.n2, nk);
    const size_t lds = rb_xz_lds(g);
    const int xc = rb_xc(g);
    const double *thd = static_cast<const double *>(thv);
#define LTD_XZ(a, c) hipLaunchKernelGGL((k_rb_xz<a, c>), grid, block, lds, s, g, ka, ncols, xc, thd)
    if (g.n1 == 16 && g.n3 == 16) LTD_XZ(16, 16);
    else if (g.n1 == 64 && g.n3 == 64) LTD_XZ(64, 64);
    else if (g.n1 == 72 && g.n3 == 72) LTD_XZ(72, 72);
    else if (g.n1 == 96 && g.n3 == 160) LTD_XZ(96, 160);
    else LTD_XZ(0, 0);
#undef LTD_XZ
  } else {
    const dim3 grid(g.nbz, ncols, nk);
    const size_t lds = rb_cache_lds(g, fp32 ? sizeof(float2) : sizeof(double2));
#define LTD_RY(a)                                                                 \
  do {                                                                            \
    if (fp32) hipLaunchKernelGGL((k_rb_y<a, float2>), grid, block, lds, s, g, ka, ncols); \
    else hipLaunchKernelGGL((k_rb_y<a, double2>), grid, block, lds, s, g, ka, ncols);     \
  } while (0)
    if (g.n2 == 64 && g.nbx <= 32 && g.by <= 15) {
      const size_t lds64 = y64_lds_bytes();
      if (fp32) hipLaunchKernelGGL(k_rb_y64<float2>, grid, dim3(256), lds64, s, g, ka, ncols);
      else hipLaunchKernelGGL(k_rb_y64<double2>, grid, dim3(256), lds64, s, g, ka, ncols);
    } else if (g.n2 == 72 && g.nbx <= Y72_LINES) {
      const size_t l72 = y72_lds_bytes(g, fp32 ? sizeof(float2) : sizeof(double2));
      const bool pr = 4 * g.by + 1 <= 72;
      if (fp32) {
        if (pr) hipLaunchKernelGGL((k_rb_y72<float2, true>), grid, dim3(320), l72, s, g, ka, ncols);
        else hipLaunchKernelGGL((k_rb_y72<float2, false>), grid, dim3(320), l72, s, g, ka, ncols);
      } else {
        if (pr) hipLaunchKernelGGL((k_rb_y72<double2, true>), grid, dim3(320), l72, s, g, ka, ncols);
        else hipLaunchKernelGGL((k_rb_y72<double2, false>), grid, dim3(320), l72, s, g, ka, ncols);
      }
    } else if (g.n2 == 16) LTD_RY(16);
    else if (g.n2 == 64) LTD_RY(64);
    else if (g.n2 == 72) LTD_RY(72);
    else if (g.n2 == 96) LTD_RY(96);
    else LTD_RY(0);
#undef LTD_RY
  }
  return hipGetLastError();
}

size_t fft_plane_lds_bytes(const Grid &g) { return plane_lds(g); }
size_t fft_line_lds_bytes(const Grid &g) { return line_lds(g, line_tile(g, false), false); }

// the register plane passes: square 72- or 64-point planes, box within the exact-grid bound
bool plane_reg_ok(const Grid &g);

bool fft_ap_box_ok(const Grid &g) { return plane_reg_ok(g) && rb_fast(g); }

hipError_t fft_ap_inverse_y(const Grid &g, const FftKArgs &ka, int ncols, int nfields, hipStream_t s) {
  set_attrs();
  if (!fft_ap_box_ok(g)) return hipErrorInvalidValue;
  const dim3 grid(g.nbz, ncols, 1);
  const size_t lds = (size_t)g.nbx * rb_pitch(g.n2) * sizeof(double2);
  if (g.n2 == 72) hipLaunchKernelGGL(k_ap_inv_y<72>, grid, dim3(256), lds, s, g, ka, ncols, nfields);
  else hipLaunchKernelGGL(k_ap_inv_y<64>, grid, dim3(256), lds, s, g, ka, ncols, nfields);
  return hipGetLastError();
}

hipError_t fft_ap_combine(const FwdOut &fo, const KSphere &sp, const double2 *ys, int ncols, int mode, double alpha_a,
                          double beta_a, hipStream_t s) {
  const long long tot = (long long)sp.n_g * ncols;
  const int nb = (int)std::min<long long>((tot + 255) / 256, 16384);
  if (mode == FFT_MODE_V)
    hipLaunchKernelGGL(k_ap_combine<FFT_MODE_V>, dim3(nb), dim3(256), 0, s, fo, sp, ys, ncols, alpha_a, beta_a);
  else if (mode == FFT_MODE_HS)
    hipLaunchKernelGGL(k_ap_combine<FFT_MODE_HS>, dim3(nb), dim3(256), 0, s, fo, sp, ys, ncols, alpha_a, beta_a);
  else
    hipLaunchKernelGGL(k_ap_combine<FFT_MODE_TVPS>, dim3(nb), dim3(256), 0, s, fo, sp, ys, ncols, alpha_a, beta_a);
  return hipGetLastError();
}

bool plane_reg_ok(const Grid &g) {
  return g.n1 == g.n2 && (g.n1 == 72 || g.n1 == 64) && 4 * g.bx + 1 <= g.n1 && 4 * g.by + 1 <= g.n2;
}

hipError_t fft_inverse_planes(const Grid &g, const FftKArgs &ka, int nk, int ncols, int nfields, hipStream_t s) {
  set_attrs();
  const dim3 grid(g.nbz, ncols, nk), block(FFT_NT);
  if (plane_reg_ok(g)) {
    if (g.n1 == 72)
      hipLaunchKernelGGL(k_inv_plane_reg<72>, grid, dim3(256), plane_reg_lds<72>(g.nbx), s, g, ka, ncols, nfields);
    else
      hipLaunchKernelGGL(k_inv_plane_reg<64>, grid, dim3(256), plane_reg_lds<64>(g.nbx), s, g, ka, ncols, nfields);
    return hipGetLastError();
  }
  const size_t lds = plane_lds(g);
#define LTD_INV(a, b) hipLaunchKernelGGL((k_inv_plane<a, b>), grid, block, lds, s, g, ka, ncols, nfields, plane_ch(g))
  if (g.n1 == 16 && g.n2 == 16) LTD_INV(16, 16);
  else if (g.n1 == 64 && g.n2 == 64) LTD_INV(64, 64);
  else if (g.n1 == 72 && g.n2 == 72) LTD_INV(72, 72);
  else if (g.n1 == 96 && g.n2 == 96) LTD_INV(96, 96);
  else LTD_INV(0, 0);
#undef LTD_INV
  return hipGetLastError();
}

hipError_t fft_lines(const Grid &g, const FftKArgs &ka, int nk, int ncols, int mode, const double *thv,
                     hipStream_t s) {
  set_attrs();
  const bool vmode = (mode == FFT_MODE_V);
  // register line transforms where the length has a two-factor split and the
  // box fits the exact-grid bound (64 = 8 x 8, 72 = 8 x 9, 108 = 12 x 9)
  if (4 * g.bz + 1 <= g.n3 && (g.n3 == 64 || g.n3 == 72 || g.n3 == 108)) {
#define LTD_LR(nz, z1)                                                                                   \
  do {                                                                                                   \
    using TZ = Two<nz, z1, nz / z1>;                                                                     \
    constexpr int LZ = rb_lz(TZ::LPW);                                                                   \
    const long long pl = (long long)g.n1 * g.n2;                                                         \
    const dim3 gr((unsigned)((pl + 4 * LZ - 1) / (4 * LZ)), ncols, nk);                                  \
    const size_t lds = (size_t)4 * LZ * XchPitch<nz, z1>::LS * sizeof(double);                           \
    if (vmode) hipLaunchKernelGGL((k_lines_reg<nz, z1, true>), gr, dim3(256), lds, s, g, ka, ncols, thv); \
    else hipLaunchKernelGGL((k_lines_reg<nz, z1, false>), gr, dim3(256), lds, s, g, ka, ncols, thv);     \
  } while (0)
    if (g.n3 == 64) LTD_LR(64, 8);
    else if (g.n3 == 72) LTD_LR(72, 8);
    else LTD_LR(108, 12);
#undef LTD_LR
    return hipGetLastError();
  }
  const int t = line_tile(g, vmode);
  const long long plane_sz = (long long)g.n1 * g.n2;
  const int ntile = (int)((plane_sz + t - 1) / t);
  const dim3 grid(ntile, ncols, nk), block(FFT_NT);
  const size_t lds = line_lds(g, t, vmode);
#define LTD_LN(a)                                                                               \
  if (vmode) hipLaunchKernelGGL((k_lines<a, true>), grid, block, lds, s, g, ka, ncols, t, thv); \
  else hipLaunchKernelGGL((k_lines<a, false>), grid, block, lds, s, g, ka, ncols, t, thv)
  if (g.n3 == 16) {
    LTD_LN(16);
  } else if (g.n3 == 64) {
    LTD_LN(64);
  } else if (g.n3 == 72) {
    LTD_LN(72);
  } else if (g.n3 == 108) {
    LTD_LN(108);
  } else if (g.n3 == 160) {
    LTD_LN(160);
  } else {
    LTD_LN(0);
  }
#undef LTD_LN
  return hipGetLastError();
}

hipError_t fft_forward_planes(const Grid &g, const FftKArgs &ka, int nk, int ncols, int mode, double alpha_a,
                              double beta_a, hipStream_t s) {
  set_attrs();
  const dim3 grid(g.nbz, ncols, nk), block(FFT_NT);
  if (plane_reg_ok(g)) {
#define LTD_FR(a, m) \
  hipLaunchKernelGGL((k_fwd_plane_reg<a, m>), grid, dim3(256), plane_reg_lds<a>(g.nbx), s, g, ka, ncols, alpha_a, beta_a)
#define LTD_FRM(a)                                   \
  do {                                               \
    if (mode == FFT_MODE_V) LTD_FR(a, FFT_MODE_V);   \
    else if (mode == FFT_MODE_HS) LTD_FR(a, FFT_MODE_HS); \
    else LTD_FR(a, FFT_MODE_TVPS);                   \
  } while (0)
    if (g.n1 == 72) LTD_FRM(72);
    else LTD_FRM(64);
#undef LTD_FRM
#undef LTD_FR
    return hipGetLastError();
  }
  const size_t lds = plane_lds(g);
#define LTD_FW(a, b) \
  hipLaunchKernelGGL((k_fwd_plane<a, b>), grid, block, lds, s, g, ka, ncols, mode, alpha_a, beta_a, plane_ch(g))
  if (g.n1 == 16 && g.n2 == 16) LTD_FW(16, 16);
  else if (g.n1 == 64 && g.n2 == 64) LTD_FW(64, 64);
  else if (g.n1 == 72 && g.n2 == 72) LTD_FW(72, 72);
  else if (g.n1 == 96 && g.n2 == 96) LTD_FW(96, 96);
  else LTD_FW(0, 0);
#undef LTD_FW
  return hipGetLastError();
}

}  // namespace ltd
