// C-ABI of the ltd library: validation, workspace planning and the
// orchestration of the kernels for the LAPW+LO operator applies, the subspace
// set-up and the time step (Pela & Draxl, Secs. 2.1-2.3, App. A).
#include "ltd.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <unordered_set>
#include <vector>

#include "common.h"
#include "subspace.h"

using namespace ltd;

namespace {

constexpr size_t ALIGN = 256;
constexpr long long PART_TILES = 2048;  // split-K partial budget (64x64 complex tiles)
// launches of the x/z kernel per timed step stage (the stage is their mean)
constexpr int PROF_XZ_REPS = 4;
// steps captured per graph: a call replays the largest that fit, then the smaller ones
constexpr int GRAPH_TIERS = 3;
constexpr int GRAPH_STEPS[GRAPH_TIERS] = {32, 8, 1};

size_t up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

struct Arena {
  size_t off = 0;
  size_t take(size_t bytes) {
    const size_t o = off;
    off += up(bytes);
    return o;
  }
};

// One entry of the K2 (block-diagonal muffin-tin) problem tables.
struct K2Table {
  std::vector<ZProb> p1, p2;  // first pass (beta = 0), second pass (beta = 1)
  int tiles1 = 0, tiles2 = 0;
  size_t off1 = 0, off2 = 0;  // device offsets of the tables in the workspace
  bool built = false;
};

struct KHost {
  int n_g, n_basis, k_ext;
  size_t g_off;            // first G of this k in the concatenated arrays
  size_t amat_off;         // element offset of A_k
  std::vector<int> plane_ptr, pts_g, pts_xy, pts_xy_a, plane_x;
  size_t o_ptsxy_a = 0, o_pxr = 0;
  // workspace offsets
  size_t o_gk, o_pptr, o_ptsg, o_ptsxy;
  size_t o_subs;           // Tsub, Vsub, Psub, Ssub (4 n^2, Phi basis)
  size_t o_tilde;          // Tt, Vt_ref, Pt (3 n^2), then H0t (n^2)
  size_t o_L, o_Linv, o_LH, o_LinvH, o_vstep, o_work, o_hm, o_dev;
  size_t o_phit, o_yext, o_cache;
  size_t o_phit32 = 0, o_yext32 = 0;  // FP32 residual: complex64 Phi~_ext (atom-contiguous MT rows) and Y_ext
  // matrix-matrix route: G triples on the device and the dense interstitial
  // blocks T, V (reference potential), P_z, S (natural G order) and V of the step
  // (sphere-table order, the row order of Phi~_ext)
  size_t o_gint = 0, o_mmT = 0, o_mmV = 0, o_mmP = 0, o_mmS = 0, o_mmVt = 0;
  // bound subspace
  bool bound = false;
  const double2 *phi = nullptr;
  int ldphi = 0;
  double lam_min = 0, lam_max = 0;
};

}  // namespace

struct ltd_system {
  // description
  int n_k = 0;
  std::vector<KHost> kh;
  std::vector<int32_t> g_int;
  std::vector<double> gk;
  int n1 = 0, n2 = 0, n3 = 0;
  long long ngrid = 0;
  const double *theta = nullptr, *v_r = nullptr;
  int n_atoms = 0;
  std::vector<int> n_mt, n_lo, a_off, l_off, s_off;
  int n_a = 0, n_lo_tot = 0, n_loc = 0;
  long long blk_elems = 0;  // sum s_a^2
  const double2 *amat = nullptr, *h = nullptr, *o = nullptr, *pz = nullptr;
  double omega = 0, c_light = 0, occ = 0;
  std::vector<double> kw;
  int n_aux = 0, n_states = 0, max_cols = 0, precision = 0;
  int route = LTD_ROUTE_FFT;  // interstitial route
  size_t o_box_t = 0, o_box_v = 0, o_box_step = 0, o_box_scr = 0;  // MM: Fourier coefficient boxes
  int nb_max = 0;
  // grid plan; rgrid: the grid of the per-step rebuild (same box, lengths
  // >= 4 b + 1), with W synthesised from Theta V when it is smaller
  Grid grid{};
  Grid rgrid{};
  bool rb_synth = false;
  // the FFT-route apply on the rebuild grid (exact: the products it forms need
  // Theta~ and (Theta V)~ only at differences of two box frequencies), with
  // Theta and Theta V synthesised there in grid order and sphere tables in its
  // coordinates
  bool ap_red = false;
  size_t o_th_ap = 0, o_thv_ap = 0, o_ones = 0;
  // the apply's box route (register x/z and y kernels of the rebuild on the apply
  // grid): Theta and Theta V of the bound potential in the x/z kernel's layout
  bool ap_box = false;
  bool planes_only = false;  // LTD_ROUTE_FFT_PLANES: never the box route
  size_t o_th_x = 0, o_thv_x = 0;
  int rb_variant = 0;      // launch shape of the x/z rebuild kernel (tuned)
  int vproj_target = 512;  // block target of the projection GEMM's K split (tuned)
  // side stream of the rebuild: the muffin-tin branch runs beside the FFT chain
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // pipelined propagation: the exponential of step n on `side2` beside the
  // rebuild of step n + 1 (ev_p0: step start, ev_asm: H~(mid) assembled, ev_pj: step done)
  hipStream_t side2 = nullptr;
  hipEvent_t ev_p0 = nullptr, ev_asm = nullptr, ev_pj = nullptr;
  // and Theta V of step n + 1 synthesised on `side3` into the buffer step n does
  // not read, beside its x/z transforms (or, when both are the same buffer, once
  // they have read it: ev_xz), done before its y transforms (ev_syn)
  hipStream_t side3 = nullptr;
  hipEvent_t ev_xz = nullptr, ev_syn = nullptr;
  size_t o_rtw1 = 0, o_rtw2 = 0, o_rtw3 = 0, o_M1 = 0, o_M2 = 0, o_M3 = 0, o_syn1 = 0, o_syn2 = 0;
  size_t o_F1 = 0, o_F2 = 0, o_F3 = 0;  // MFMA fragments of the synthesis axis matrices
  int chunk = 0;        // columns per apply pass
  bool h_in_lds = false;
  bool p_in_lds = false;
  // workspace
  char *ws = nullptr;
  size_t ws_need = 0, ws_bound = 0;
  size_t o_tw1, o_tw2, o_tw3, o_thv, o_thv_rb, o_thv_step, o_status, o_part, o_partials;
  size_t o_thv_step2 = 0;  // second Theta V buffer of the pipelined rebuild (steps of odd index in a graph)
  size_t o_vpartials;  // split-K partials of the V~ projection (its own: reduced on another stream)
  size_t o_slab_in, o_slab_out, o_W, o_Y, o_heff, o_tvps, o_proj, o_tmp3, o_eigA, o_eigV, o_eigw, o_eigwork;
  size_t o_stepslab, o_subdev, o_theta_sc, o_k6, o_hstep, o_zero32;
  K2Table k2_hs, k2_tvps, k2_step;
  size_t o_k2_hs1, o_k2_hs2, o_k2_tv1, o_k2_tv2, o_k2_st1, o_k2_st2;
  std::vector<ZProb> vstep_tab;
  int vstep_tiles = 0;
  size_t o_vstep_tab;
  // FP32 residual: the block products (complex64 blocks h(t) - h, FP32 matrix
  // cores) and the projection on complex64 operands; MT rows permuted so that
  // each atom's channels and local orbitals are contiguous (mtperm: FP64 row of
  // each FP32 row, relative to N_G)
  std::vector<ZProb> k7_32, vstep32;
  int k7_32_tiles = 0, vstep32_tiles = 0;
  size_t o_k7_32 = 0, o_vstep32 = 0, o_hstep32 = 0, o_mtperm = 0;
  size_t o_full = 0, o_fscal = 0;  // full-basis propagation: eight N_basis x cols blocks, CG scalars
  std::vector<int> mt_row32;  // first FP32 MT row of each atom
  const void *k2_step_h = nullptr;  // blocks the step table points at
  // subspace / step state
  std::vector<SubDev> sd;
  double cheb_dt = NAN;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t gexec[GRAPH_TIERS] = {};  // GRAPH_STEPS[t] steps per replay
  hipGraph_t graph[GRAPH_TIERS] = {};
  ltd_step_args gargs{};
  bool gvalid = false;
  bool gpipe = false;  // the captured step is the pipelined one

  template <class T>
  T *at(size_t off) const {
    return reinterpret_cast<T *>(ws + off);
  }
};

namespace {

#define LTD_HIP(x)                      \
  do {                                  \
    hipError_t e_ = (x);                \
    if (e_ != hipSuccess) return LTD_EHIP; \
  } while (0)

#define LTD_TRY(x)                  \
  do {                              \
    ltd_status s_ = (x);            \
    if (s_ != LTD_OK) return s_;    \
  } while (0)

hipStream_t S(void *s) { return reinterpret_cast<hipStream_t>(s); }

// Stage timer: records an event after each stage on the stream (eager runs only).
struct Prof {
  hipStream_t s = nullptr;
  std::vector<hipEvent_t> ev;
  std::vector<int> tag;
  ltd_status begin(hipStream_t st) {
    s = st;
    hipEvent_t e;
    LTD_HIP(hipEventCreate(&e));
    LTD_HIP(hipEventRecord(e, s));
    ev.push_back(e);
    tag.push_back(-1);
    return LTD_OK;
  }
  ltd_status mark(int stage) {
    hipEvent_t e;
    LTD_HIP(hipEventCreate(&e));
    LTD_HIP(hipEventRecord(e, s));
    ev.push_back(e);
    tag.push_back(stage);
    return LTD_OK;
  }
  // adds elapsed ms per stage into acc; destroys the events
  ltd_status collect(double *acc, int nstage) {
    LTD_HIP(hipEventSynchronize(ev.back()));
    for (size_t i = 1; i < ev.size(); ++i) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev[i - 1], ev[i]) != hipSuccess) ms = 0.f;
      if (tag[i] >= 0 && tag[i] < nstage) acc[tag[i]] += ms;
    }
    for (auto e : ev) (void)hipEventDestroy(e);
    ev.clear();
    tag.clear();
    return LTD_OK;
  }
};

#define LTD_MARK(p, st)                 \
  do {                                  \
    if (p) LTD_TRY((p)->mark(st));      \
  } while (0)

// ---------------------------------------------------------------------------
// Bessel functions J_0..J_nmax(x) by Miller's backward recurrence, normalised
// with J_0 + 2 sum_k J_2k = 1.
// ---------------------------------------------------------------------------
void bessel_j(double x, int nmax, std::vector<double> &out) {
  out.assign(nmax + 1, 0.0);
  if (x == 0.0) {
    out[0] = 1.0;
    return;
  }
  const double ax = std::fabs(x);
  const int top = std::max(nmax, (int)std::ceil(ax));
  int m = top + 30 + (int)std::sqrt(40.0 * top);
  if (m % 2) ++m;
  std::vector<double> t(m + 2, 0.0);
  t[m] = 1e-30;
  for (int k = m; k >= 1; --k) {
    t[k - 1] = (2.0 * k / ax) * t[k] - t[k + 1];
    if (std::fabs(t[k - 1]) > 1e250)
      for (int q = k - 1; q <= m; ++q) t[q] *= 1e-250;
  }
  double norm = t[0];
  for (int k = 2; k <= m; k += 2) norm += 2.0 * t[k];
  for (int k = 0; k <= nmax; ++k) {
    double v = t[k] / norm;
    if (x < 0 && (k % 2)) v = -v;  // J_k(-x) = (-1)^k J_k(x)
    out[k] = v;
  }
}

// exp(-i tau x) = sum_k c_k T_k(x); returns the degree (or -1 if kmax is too small).
int cheb_coef(double tau, int kmax, std::vector<double2> &c) {
  std::vector<double> j;
  bessel_j(tau, kmax + 2, j);
  c.assign(kmax + 1, make_double2(0.0, 0.0));
  int deg = -1;
  for (int k = 0; k <= kmax; ++k) {
    const double a = (k == 0 ? 1.0 : 2.0) * j[k];
    // (-i)^k
    const int r = k % 4;
    c[k] = (r == 0) ? make_double2(a, 0.0) : (r == 1) ? make_double2(0.0, -a) : (r == 2) ? make_double2(-a, 0.0)
                                                                                      : make_double2(0.0, a);
  }
  for (int k = 1; k <= kmax; ++k) {
    if (k > std::fabs(tau) && std::fabs(j[k]) + std::fabs(j[k + 1]) + std::fabs(j[k + 2]) < 1e-18) {
      deg = k;
      break;
    }
  }
  return deg;
}

// ---------------------------------------------------------------------------
// GEMM helpers
// ---------------------------------------------------------------------------
ZProb zp(int m, int n, int k, const double2 *A, int lda, const double2 *B, int ldb, double2 *C, int ldc,
         double2 alpha = make_double2(1.0, 0.0), double2 beta = make_double2(0.0, 0.0), int batch = 1,
         long long sA = 0, long long sB = 0, long long sC = 0) {
  ZProb p{};
  p.A = A;
  p.B = B;
  p.C = C;
  p.lda = lda;
  p.ldb = ldb;
  p.ldc = ldc;
  p.m = m;
  p.n = n;
  p.k = k;
  p.batch = batch;
  p.sA = sA;
  p.sB = sB;
  p.sC = sC;
  p.alpha = alpha;
  p.beta = beta;
  return p;
}

// problems held by value, GEMM_MAXP per launch; K split within part_tiles partial
// tiles (64 x 64 complex) of the buffer part
ltd_status gemm_buf(int opa, int opb, const std::vector<ZProb> &probs, double2 *part, long long part_tiles,
                    hipStream_t s) {
  for (size_t i0 = 0; i0 < probs.size(); i0 += GEMM_MAXP) {
    ZBatch b{};
    b.nprob = (int)std::min<size_t>(GEMM_MAXP, probs.size() - i0);
    for (int i = 0; i < b.nprob; ++i) b.p[i] = probs[i0 + i];
    gemm_plan(b.p, b.nprob, &b.total_tiles, 512, part_tiles);
    LTD_HIP(gemm_launch(opa, opb, b, part, s));
  }
  return LTD_OK;
}

ltd_status gemm(ltd_system *sys, int opa, int opb, std::vector<ZProb> probs, hipStream_t s) {
  return gemm_buf(opa, opb, probs, sys->at<double2>(sys->o_partials), PART_TILES, s);
}

ltd_status gemm1(ltd_system *sys, int opa, int opb, const ZProb &p, hipStream_t s) {
  return gemm(sys, opa, opb, std::vector<ZProb>{p}, s);
}

// K2 tables: Y_x = blockdiag(x_a) W for every atom a and matrix x in `xs`.  The
// local vector of atom a is [W rows of its channels; W rows of its LOs] (two row
// segments of W), so each output block is one GEMM over a two-segment K.
void build_k2(const ltd_system *sys, const std::vector<const double2 *> &xs, const double2 *W, int ldw,
              const std::vector<double2 *> &Ys, int ldy, int cols, std::vector<ZProb> &p1, std::vector<ZProb> &p2) {
  const double2 one = make_double2(1.0, 0.0), zero = make_double2(0.0, 0.0);
  (void)p2;
  for (size_t xi = 0; xi < xs.size(); ++xi) {
    for (int a = 0; a < sys->n_atoms; ++a) {
      const int m = sys->n_mt[a], l = sys->n_lo[a], s = m + l;
      const double2 *x = xs[xi] + sys->s_off[a];
      const double2 *wt = W + sys->a_off[a];
      const double2 *wl = W + sys->n_a + sys->l_off[a];
      double2 *yt = Ys[xi] + sys->a_off[a];
      double2 *yl = Ys[xi] + sys->n_a + sys->l_off[a];
      ZProb top = zp(m, cols, s, x, s, wt, ldw, yt, ldy, one, zero);
      top.B2 = wl;
      top.kseg = l > 0 ? m : 0;
      p1.push_back(top);
      if (l > 0) {
        ZProb bot = zp(l, cols, s, x + m, s, wt, ldw, yl, ldy, one, zero);
        bot.B2 = wl;
        bot.kseg = m;
        p1.push_back(bot);
      }
    }
  }
}

// target: the planner's block target (K is split below it; 0: never split)
ltd_status upload_k2(ltd_system *sys, std::vector<ZProb> &p1, std::vector<ZProb> &p2, K2Table &t, size_t off1,
                     size_t off2, size_t cap, int target = 512) {
  int tt = 0;
  gemm_plan(p1.data(), (int)p1.size(), &tt, target, PART_TILES);
  t.tiles1 = tt;
  tt = 0;
  if (!p2.empty()) gemm_plan(p2.data(), (int)p2.size(), &tt, 512, PART_TILES);
  t.tiles2 = tt;
  if (p1.size() * sizeof(ZProb) > cap || p2.size() * sizeof(ZProb) > cap) return LTD_EUNSUPPORTED;
  t.p1 = p1;
  t.p2 = p2;
  t.off1 = off1;
  t.off2 = off2;
  LTD_HIP(hipMemcpy(sys->ws + off1, p1.data(), p1.size() * sizeof(ZProb), hipMemcpyHostToDevice));
  if (!p2.empty()) LTD_HIP(hipMemcpy(sys->ws + off2, p2.data(), p2.size() * sizeof(ZProb), hipMemcpyHostToDevice));
  t.built = true;
  return LTD_OK;
}

ltd_status run_k2(ltd_system *sys, const K2Table &t, int cols, hipStream_t s) {
  if (!t.p1.empty())
    LTD_HIP(gemm_launch_table(OP_N, OP_N, sys->at<ZProb>(t.off1), t.p1.data(), (int)t.p1.size(), t.tiles1,
                              sys->at<double2>(sys->o_partials), cols, s));
  if (!t.p2.empty())
    LTD_HIP(gemm_launch_table(OP_N, OP_N, sys->at<ZProb>(t.off2), t.p2.data(), (int)t.p2.size(), t.tiles2,
                              sys->at<double2>(sys->o_partials), cols, s));
  return LTD_OK;
}

// ---------------------------------------------------------------------------
// FFT argument helpers
// ---------------------------------------------------------------------------
KSphere sphere_of(const ltd_system *sys, int k) {
  const KHost &h = sys->kh[k];
  KSphere sp{};
  sp.gk = sys->at<double>(h.o_gk);
  sp.plane_ptr = sys->at<int>(h.o_pptr);
  sp.pts_g = sys->at<int>(h.o_ptsg);
  sp.pts_xy = sys->at<int>(h.o_ptsxy);
  sp.plane_x = sys->at<int>(h.o_pxr);
  sp.n_g = h.n_g;
  return sp;
}

// grid, sphere tables and Theta V of the apply's interstitial passes
KSphere sphere_ap(const ltd_system *sys, int k) {
  KSphere sp = sphere_of(sys, k);
  if (sys->ap_red) sp.pts_xy = sys->at<int>(sys->kh[k].o_ptsxy_a);
  return sp;
}

// bytes per value of the rebuild cache and step slabs (complex64 for the FP32 residual)
size_t rb_elem(const ltd_system *sys) {
  return sys->precision == LTD_FP32_RESID ? sizeof(float2) : sizeof(double2);
}

Grid grid_of(const ltd_system *sys) {
  Grid g = sys->grid;
  g.tw1 = sys->at<double2>(sys->o_tw1);
  g.tw2 = sys->at<double2>(sys->o_tw2);
  g.tw3 = sys->at<double2>(sys->o_tw3);
  g.theta = sys->theta;
  return g;
}

// grid of the per-step rebuild
Grid rgrid_of(const ltd_system *sys) {
  if (!sys->rb_synth) return grid_of(sys);
  Grid g = sys->rgrid;
  g.tw1 = sys->at<double2>(sys->o_rtw1);
  g.tw2 = sys->at<double2>(sys->o_rtw2);
  g.tw3 = sys->at<double2>(sys->o_rtw3);
  g.theta = sys->theta;
  return g;
}

bool resid32(const ltd_system *sys) { return sys->precision == LTD_FP32_RESID; }

Grid agrid_of(const ltd_system *sys) {
  if (!sys->ap_red) return grid_of(sys);
  Grid g = rgrid_of(sys);
  g.theta = sys->at<double>(sys->o_th_ap);
  return g;
}
const double *athv_of(const ltd_system *sys) {
  return sys->at<double>(sys->ap_red ? sys->o_thv_ap : sys->o_thv);
}

// Theta v in the layout of the rebuild step (W on the rebuild grid when it is
// smaller); v read at v + (*step) * stride when step is not NULL.  resid: the
// difference from the reference, W(t) - W_ref or Theta (v - v_ref), in FP32.
ltd_status rebuild_potential(ltd_system *sys, const double *v, const int *step, long long stride, void *out,
                             bool resid, hipStream_t s) {
  if (sys->rb_synth) {
    LTD_HIP(fft_rb_synth(rgrid_of(sys), sys->n1, sys->n2, sys->n3, sys->theta, v, step, stride,
                         sys->at<double>(sys->o_M1), sys->at<double>(sys->o_M2), sys->at<double>(sys->o_M3),
                         sys->at<double>(sys->o_F1), sys->at<double>(sys->o_F2), sys->at<double>(sys->o_F3),
                         sys->at<double>(sys->o_syn1), sys->at<double>(sys->o_syn2), out,
                         resid ? sys->at<double>(sys->o_thv_rb) : nullptr, resid, s));
  } else {
    LTD_HIP(fft_rb_thv(grid_of(sys), sys->theta, v, step, stride, out, resid ? sys->v_r : nullptr, resid, s));
  }
  return LTD_OK;
}

// the blocks the muffin-tin step table reads: a per-step series goes through
// a fixed copy buffer, one set of blocks is read in place (NULL: the reference)
const void *k2_source(const ltd_system *sys, const ltd_step_args *a) {
  if (resid32(sys)) return sys->at<double2>(sys->o_hstep);  // the block difference h(t) - h
  if (!a->h_t) return nullptr;
  return a->h_stride ? static_cast<const void *>(sys->at<double2>(sys->o_hstep)) : a->h_t;
}

// ---------------------------------------------------------------------------
// Operator apply on a column chunk of one k-point.
//   mode FFT_MODE_HS:   out[0] = H(A) C, out[1] = S C
//   mode FFT_MODE_TVPS: out[0..3] = T C, V C, P_z C, S C
// ---------------------------------------------------------------------------
// Apply stages (profiling tags): 0 inverse planes, 1 z lines, 2 forward planes,
// 3 A C (K1), 4 block-diagonal muffin-tin products (K2), 5 A^H Y (K3) and LO rows.
// Scratch of one apply pass: FFT slabs (4 input and 5 output fields), the
// muffin-tin vectors W and products Y (blocks ystride apart), the effective
// blocks h + (A/c) p_z + (A^2/2c^2) o, and the GEMMs' split-K partials.
// k2_tables: the block products come from the tables uploaded at bind, which
// point at the workspace's W and Y; otherwise they are passed by value.
struct ApplyBufs {
  double2 *slab_in, *slab_out, *W, *Y, *heff, *part;
  long long ystride, part_tiles;
  bool k2_tables;
};

ltd_status apply_mt(ltd_system *sys, int k, int mode, double al, double be, const double2 *C, int ldc, int cols,
                    double2 *const out[4], const int ldo[4], hipStream_t s, Prof *pf, const ApplyBufs &bf);

// Interstitial part of an apply by the dense blocks: HS mode H(A) C = T C + V C +
// (A/c) P C + (A^2/2c^2) S C and S C; TVPS mode T C, V C, P C, S C (plane-wave
// rows of out, overwritten).  Problems that add into one output run in
// successive launches.
ltd_status apply_mm(ltd_system *sys, int k, int mode, double al, double be, const double2 *C, int ldc, int cols,
                    double2 *const out[4], const int ldo[4], const ApplyBufs &bf, hipStream_t s) {
  const KHost &kh = sys->kh[k];
  const int ng = kh.n_g;
  const double2 one = make_double2(1.0, 0.0), zero = make_double2(0.0, 0.0);
  const auto blk = [&](size_t off) { return sys->at<double2>(off); };
  if (mode == FFT_MODE_TVPS) {
    const size_t m[4] = {kh.o_mmT, kh.o_mmV, kh.o_mmP, kh.o_mmS};
    std::vector<ZProb> p;
    for (int x = 0; x < 4; ++x) p.push_back(zp(ng, cols, ng, blk(m[x]), ng, C, ldc, out[x], ldo[x]));
    return gemm_buf(OP_N, OP_N, p, bf.part, bf.part_tiles, s);
  }
  LTD_TRY(gemm_buf(OP_N, OP_N, {zp(ng, cols, ng, blk(kh.o_mmT), ng, C, ldc, out[0], ldo[0]),
                                zp(ng, cols, ng, blk(kh.o_mmS), ng, C, ldc, out[1], ldo[1])},
                   bf.part, bf.part_tiles, s));
  LTD_TRY(gemm_buf(OP_N, OP_N, {zp(ng, cols, ng, blk(kh.o_mmV), ng, C, ldc, out[0], ldo[0], one, one)}, bf.part,
                   bf.part_tiles, s));
  if (al != 0.0)
    LTD_TRY(gemm_buf(OP_N, OP_N, {zp(ng, cols, ng, blk(kh.o_mmP), ng, C, ldc, out[0], ldo[0], make_double2(al, 0.0),
                                     one)}, bf.part, bf.part_tiles, s));
  if (be != 0.0)
    LTD_TRY(gemm_buf(OP_N, OP_N, {zp(ng, cols, ng, blk(kh.o_mmS), ng, C, ldc, out[0], ldo[0], make_double2(be, 0.0),
                                     one)}, bf.part, bf.part_tiles, s));
  (void)zero;
  return LTD_OK;
}

ApplyBufs workspace_bufs(const ltd_system *sys) {
  ApplyBufs b{};
  b.slab_in = sys->at<double2>(sys->o_slab_in);
  b.slab_out = sys->at<double2>(sys->o_slab_out);
  b.W = sys->at<double2>(sys->o_W);
  b.Y = sys->at<double2>(sys->o_Y);
  b.heff = sys->at<double2>(sys->o_heff);
  b.part = sys->at<double2>(sys->o_partials);
  b.ystride = (long long)sys->n_loc * sys->chunk;
  b.part_tiles = PART_TILES;
  b.k2_tables = true;
  return b;
}

// Interstitial part of an apply by the box route: the y images of the input
// fields (psi, and pi_x, pi_y, pi_z unless MODE_V), the rebuild's x/z kernel
// once per (input field, multiplier) pass with the fields as pseudo k-points
// (psi Theta, pi_i Theta into fields 0, 2, 3, 4; psi Theta V into field 1), its
// y kernel (sphere order, into slab_in: the y images are read by then) and the
// mode's combination.  The slabs hold box arrays (nbz x N2 x nbx per column and
// field) instead of whole planes.
ltd_status apply_box(ltd_system *sys, int k, int mode, double al, double be, const double2 *C, int ldc, int cols,
                     double2 *const out[4], const int ldo[4], const ApplyBufs &bf, hipStream_t s) {
  const Grid g = agrid_of(sys);
  const KSphere sp = sphere_ap(sys, k);
  const long long bsz = (long long)g.nbz * g.n2 * g.nbx * cols;  // one field's box slab
  const bool vm = mode == FFT_MODE_V;
  // the five sphere-order fields reuse slab_in (four plane fields per column)
  if (5LL * sp.n_g > 4LL * g.nbz * g.n1 * g.n2) return LTD_EUNSUPPORTED;
  FftKArgs ka{};
  ka.sph[0] = sp;
  ka.in[0].c = C;
  ka.in[0].ldc = ldc;
  ka.slab_out[0] = bf.slab_in;
  LTD_HIP(fft_ap_inverse_y(g, ka, cols, vm ? 1 : 4, s));
  const double *th = sys->at<double>(sys->o_th_x);
  const double *thv = sys->at<double>(sys->ap_red ? sys->o_thv_x : sys->o_thv_rb);
  const int np = vm ? 1 : 4, fout[4] = {0, 2, 3, 4};
  FftKArgs kx{};
  for (int i = 0; i < np; ++i) {
    kx.sph[i] = sp;
    kx.slab_in[i] = bf.slab_in + i * bsz;
    kx.slab_out[i] = bf.slab_out + fout[i] * bsz;
  }
  LTD_HIP(fft_rb_step(g, kx, np, cols, th, s, 0, false, 0));
  if (!vm) {
    FftKArgs kv{};
    kv.sph[0] = sp;
    kv.slab_in[0] = bf.slab_in;
    kv.slab_out[0] = bf.slab_out + bsz;
    LTD_HIP(fft_rb_step(g, kv, 1, cols, thv, s, 0, false, 0));
  }
  const int nf = vm ? 1 : 5;
  double2 *ys = bf.slab_in;
  // the y kernel decodes the sphere positions on the grid of the sphere tables
  // (g.d1, g.d2), as in the rebuild; the sphere order is the same
  const KSphere spy = sphere_of(sys, k);
  FftKArgs ky{};
  for (int f = 0; f < nf; ++f) {
    ky.sph[f] = spy;
    ky.slab_in[f] = bf.slab_out + f * bsz;
    ky.out[f].o0 = ys + (long long)f * sp.n_g * cols;
    ky.out[f].ld0 = sp.n_g;
  }
  LTD_HIP(fft_rb_step(g, ky, nf, cols, th, s, 1, false, 0));
  FwdOut fo{};
  fo.o0 = out[0];
  fo.ld0 = ldo[0];
  if (!vm) {
    fo.o1 = out[1];
    fo.ld1 = ldo[1];
  }
  if (mode == FFT_MODE_TVPS) {
    fo.o2 = out[2];
    fo.o3 = out[3];
    fo.ld2 = ldo[2];
    fo.ld3 = ldo[3];
  }
  LTD_HIP(fft_ap_combine(fo, sp, ys, cols, mode, al, be, s));
  return LTD_OK;
}

ltd_status apply_chunk(ltd_system *sys, int k, int mode, double a_z, const double2 *C, int ldc, int cols,
                       double2 *const out[4], const int ldo[4], hipStream_t s, Prof *pf, const ApplyBufs &bf) {
  if (cols <= 0) return LTD_OK;
  const KHost &kh = sys->kh[k];
  const Grid g = agrid_of(sys);
  const double al = a_z / sys->c_light, be = a_z * a_z / (2.0 * sys->c_light * sys->c_light);
  if (sys->route == LTD_ROUTE_MM) {  // interstitial by the dense blocks (first route)
    LTD_TRY(apply_mm(sys, k, mode, al, be, C, ldc, cols, out, ldo, bf, s));
    LTD_MARK(pf, 2);
    return apply_mt(sys, k, mode, al, be, C, ldc, cols, out, ldo, s, pf, bf);
  }
  if (sys->ap_box) {
    LTD_TRY(apply_box(sys, k, mode, al, be, C, ldc, cols, out, ldo, bf, s));
    LTD_MARK(pf, 0);
    LTD_MARK(pf, 1);
    LTD_MARK(pf, 2);
    return apply_mt(sys, k, mode, al, be, C, ldc, cols, out, ldo, s, pf, bf);
  }
  // interstitial
  FftKArgs ka{};
  ka.sph[0] = sphere_ap(sys, k);
  ka.in[0].c = C;
  ka.in[0].ldc = ldc;
  ka.slab_out[0] = bf.slab_in;
  LTD_HIP(fft_inverse_planes(g, ka, 1, cols, 4, s));
  LTD_MARK(pf, 0);
  ka.slab_in[0] = bf.slab_in;
  ka.slab_out[0] = bf.slab_out;
  LTD_HIP(fft_lines(g, ka, 1, cols, FFT_MODE_HS, athv_of(sys), s));
  LTD_MARK(pf, 1);
  ka.slab_in[0] = bf.slab_out;
  FwdOut fo{};
  fo.o0 = out[0];
  fo.o1 = out[1];
  fo.ld0 = ldo[0];
  fo.ld1 = ldo[1];
  if (mode == FFT_MODE_TVPS) {
    fo.o2 = out[2];
    fo.o3 = out[3];
    fo.ld2 = ldo[2];
    fo.ld3 = ldo[3];
  }
  ka.out[0] = fo;
  LTD_HIP(fft_forward_planes(g, ka, 1, cols, mode, al, be, s));
  LTD_MARK(pf, 2);
  return apply_mt(sys, k, mode, al, be, C, ldc, cols, out, ldo, s, pf, bf);
}

// Muffin-tin and local-orbital part of an apply (accumulated into out, whose
// plane-wave rows hold the interstitial part).
ltd_status apply_mt(ltd_system *sys, int k, int mode, double al, double be, const double2 *C, int ldc, int cols,
                    double2 *const out[4], const int ldo[4], hipStream_t s, Prof *pf, const ApplyBufs &bf) {
  const KHost &kh = sys->kh[k];
  // muffin-tin chain: W = [A C_G; C_LO]
  double2 *W = bf.W;
  double2 *Y = bf.Y;
  const int nl = sys->n_loc;
  const long long yst = bf.ystride;
  const double2 *Ak = sys->amat + kh.amat_off;
  LTD_TRY(gemm_buf(OP_N, OP_N, {zp(sys->n_a, cols, kh.n_g, Ak, sys->n_a, C, ldc, W, nl)}, bf.part, bf.part_tiles, s));
  if (sys->n_lo_tot > 0) LTD_HIP(launch_copy_rows(W + sys->n_a, nl, C + kh.n_g, ldc, sys->n_lo_tot, cols, false, s));
  LTD_MARK(pf, 3);
  const double2 one = make_double2(1.0, 0.0);
  std::vector<ZProb> k3;
  if (mode == FFT_MODE_HS) {
    LTD_HIP(launch_heff(bf.heff, sys->h, sys->pz, sys->o, al, be, sys->blk_elems, s));
    if (bf.k2_tables) {
      LTD_TRY(run_k2(sys, sys->k2_hs, cols, s));
    } else {
      std::vector<ZProb> p1, p2;
      build_k2(sys, {bf.heff, sys->o}, W, nl, {Y, Y + yst}, nl, cols, p1, p2);
      LTD_TRY(gemm_buf(OP_N, OP_N, p1, bf.part, bf.part_tiles, s));
    }
    LTD_MARK(pf, 4);
    // Y layout: [Y_heff | Y_o], each n_loc x (ystride / n_loc)
    for (int x = 0; x < 2; ++x) {
      double2 *Yx = Y + (long long)x * yst;
      k3.push_back(zp(kh.n_g, cols, sys->n_a, Ak, sys->n_a, Yx, nl, out[x], ldo[x], one, one));
    }
    LTD_TRY(gemm_buf(OP_C, OP_N, k3, bf.part, bf.part_tiles, s));
    for (int x = 0; x < 2; ++x)
      if (sys->n_lo_tot > 0)
        LTD_HIP(launch_copy_rows(out[x] + kh.n_g, ldo[x], Y + (long long)x * yst + sys->n_a, nl,
                                 sys->n_lo_tot, cols, false, s));
  } else {
    if (!bf.k2_tables) return LTD_EUNSUPPORTED;  // the four-operator apply runs on the workspace only
    LTD_TRY(run_k2(sys, sys->k2_tvps, cols, s));
    LTD_MARK(pf, 4);
    // Y layout: [Y_h | Y_p | Y_o] -> V, P, S
    for (int x = 0; x < 3; ++x) {
      double2 *Yx = Y + (long long)x * yst;
      k3.push_back(zp(kh.n_g, cols, sys->n_a, Ak, sys->n_a, Yx, nl, out[x + 1], ldo[x + 1], one, one));
    }
    LTD_TRY(gemm(sys, OP_C, OP_N, k3, s));
    if (sys->n_lo_tot > 0) {
      LTD_HIP(launch_copy_rows(out[0] + kh.n_g, ldo[0], nullptr, 0, sys->n_lo_tot, cols, true, s));
      for (int x = 0; x < 3; ++x)
        LTD_HIP(launch_copy_rows(out[x + 1] + kh.n_g, ldo[x + 1], Y + (long long)x * yst + sys->n_a, nl,
                                 sys->n_lo_tot, cols, false, s));
    }
  }
  LTD_MARK(pf, 5);
  return LTD_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free apply: the scratch of ltd_apply_HS_static is this array (one
// copy per device, held until the process ends), never the bound workspace.
// Host code uses only the device address hipGetSymbolAddress returns for it,
// looked up once per device (at bind, else at the entry point's first call).
// ---------------------------------------------------------------------------
static __device__ __align__(256) char scratch[LTD_STATIC_SCRATCH_BYTES];
constexpr int MAX_DEVICES = 64;
constexpr long long STATIC_PART_TILES = 64;  // split-K partial tiles within the scratch (4 MiB)
std::mutex g_scratch_mu;
char *g_scratch_ptr[MAX_DEVICES] = {};

// the device address of `scratch` on the current device (NULL on failure)
char *static_scratch() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
    g_scratch_ptr[dev] = static_cast<char *>(ptr);
  }
  return g_scratch_ptr[dev];
}

// Columns per pass of an apply whose scratch is the static array (0: not even one
// column fits), and the buffers of such a pass laid out from `base`.
int static_cols(const ltd_system *sys, int n) {
  const Grid &ag = sys->ap_red ? sys->rgrid : sys->grid;
  const long long slab_col = (long long)ag.nbz * ag.n1 * ag.n2;
  const size_t fixed = up((size_t)std::max<long long>(1, sys->blk_elems) * sizeof(double2)) +
                       up((size_t)STATIC_PART_TILES * 64 * 64 * sizeof(double2));
  // per column: 4 + 5 slab fields, W and two Y blocks, plus alignment slack of four arrays
  const size_t per_col = (size_t)(9 * slab_col + 3LL * sys->n_loc) * sizeof(double2);
  if (fixed + 4 * ALIGN + per_col > LTD_STATIC_SCRATCH_BYTES) return 0;
  const size_t c = (LTD_STATIC_SCRATCH_BYTES - fixed - 4 * ALIGN) / per_col;
  return (int)std::min<size_t>(c, (size_t)n);
}

ApplyBufs static_bufs(const ltd_system *sys, char *base, int cols) {
  const Grid &ag = sys->ap_red ? sys->rgrid : sys->grid;
  const long long slab_f = (long long)ag.nbz * ag.n1 * ag.n2 * cols;
  Arena ar;
  ApplyBufs b{};
  b.slab_in = reinterpret_cast<double2 *>(base + ar.take((size_t)4 * slab_f * sizeof(double2)));
  b.slab_out = reinterpret_cast<double2 *>(base + ar.take((size_t)5 * slab_f * sizeof(double2)));
  b.W = reinterpret_cast<double2 *>(base + ar.take((size_t)sys->n_loc * cols * sizeof(double2)));
  b.Y = reinterpret_cast<double2 *>(base + ar.take((size_t)2 * sys->n_loc * cols * sizeof(double2)));
  b.heff = reinterpret_cast<double2 *>(base + ar.take((size_t)std::max<long long>(1, sys->blk_elems) * sizeof(double2)));
  b.part = reinterpret_cast<double2 *>(base + ar.take((size_t)STATIC_PART_TILES * 64 * 64 * sizeof(double2)));
  b.ystride = (long long)sys->n_loc * cols;
  b.part_tiles = STATIC_PART_TILES;
  b.k2_tables = false;
  return b;
}

ltd_status apply_cols(ltd_system *sys, int k, int mode, double a_z, const double2 *C, int ldc, int n,
                      double2 *const out[4], const int ldo[4], hipStream_t s) {
  for (int j0 = 0; j0 < n; j0 += sys->chunk) {
    const int cols = std::min(sys->chunk, n - j0);
    double2 *o[4];
    for (int i = 0; i < 4; ++i) o[i] = out[i] ? out[i] + (long long)j0 * ldo[i] : nullptr;
    LTD_TRY(apply_chunk(sys, k, mode, a_z, C + (long long)j0 * ldc, ldc, cols, o, ldo, s, nullptr,
                        workspace_bufs(sys)));
  }
  return LTD_OK;
}

// ---------------------------------------------------------------------------
// Full-basis propagation helpers: S applied alone (the interstitial step
// function by the FFT V pass with Theta as the multiplier, or the dense block;
// the muffin-tin overlap blocks through the matching coefficients) and block
// conjugate gradients for S Y = B, one system per column.
// ---------------------------------------------------------------------------
double2 *full_blk(ltd_system *sys, int i) {
  const int fc = std::min(1024, std::max(sys->max_cols, sys->n_states));
  return sys->at<double2>(sys->o_full) + (size_t)i * sys->nb_max * fc;
}

ltd_status apply_s(ltd_system *sys, int k, const double2 *X, int ldx, int n, double2 *SX, int ld, hipStream_t s) {
  const KHost &kh = sys->kh[k];
  const int nl = sys->n_loc;
  const double2 one = make_double2(1.0, 0.0);
  const ApplyBufs bf = workspace_bufs(sys);
  for (int j0 = 0; j0 < n; j0 += sys->chunk) {
    const int cols = std::min(sys->chunk, n - j0);
    const double2 *x = X + (long long)j0 * ldx;
    double2 *out = SX + (long long)j0 * ld;
    if (sys->route == LTD_ROUTE_MM) {
      LTD_TRY(gemm1(sys, OP_N, OP_N, zp(kh.n_g, cols, kh.n_g, sys->at<double2>(kh.o_mmS), kh.n_g, x, ldx, out, ld),
                    s));
    } else if (sys->ap_box) {
      double2 *o[4] = {out, nullptr, nullptr, nullptr};
      const int lo[4] = {ld, 0, 0, 0};
      LTD_TRY(apply_box(sys, k, FFT_MODE_V, 0.0, 0.0, x, ldx, cols, o, lo, bf, s));
    } else {
      const Grid g = agrid_of(sys);
      FftKArgs ka{};
      ka.sph[0] = sphere_ap(sys, k);
      ka.in[0].c = x;
      ka.in[0].ldc = ldx;
      ka.slab_out[0] = bf.slab_in;
      LTD_HIP(fft_inverse_planes(g, ka, 1, cols, 1, s));
      ka.slab_in[0] = bf.slab_in;
      ka.slab_out[0] = bf.slab_out;
      LTD_HIP(fft_lines(g, ka, 1, cols, FFT_MODE_V, g.theta, s));
      ka.slab_in[0] = bf.slab_out;
      FwdOut fo{};
      fo.o0 = out;
      fo.ld0 = ld;
      ka.out[0] = fo;
      LTD_HIP(fft_forward_planes(g, ka, 1, cols, FFT_MODE_V, 0.0, 0.0, s));
    }
    const double2 *Ak = sys->amat + kh.amat_off;
    LTD_TRY(gemm1(sys, OP_N, OP_N, zp(sys->n_a, cols, kh.n_g, Ak, sys->n_a, x, ldx, bf.W, nl), s));
    if (sys->n_lo_tot > 0) LTD_HIP(launch_copy_rows(bf.W + sys->n_a, nl, x + kh.n_g, ldx, sys->n_lo_tot, cols, false, s));
    std::vector<ZProb> p1, p2;
    build_k2(sys, {sys->o}, bf.W, nl, {bf.Y}, nl, cols, p1, p2);
    LTD_TRY(gemm(sys, OP_N, OP_N, p1, s));
    LTD_TRY(gemm1(sys, OP_C, OP_N, zp(kh.n_g, cols, sys->n_a, Ak, sys->n_a, bf.Y, nl, out, ld, one, one), s));
    if (sys->n_lo_tot > 0)
      LTD_HIP(launch_copy_rows(out + kh.n_g, ld, bf.Y + sys->n_a, nl, sys->n_lo_tot, cols, false, s));
  }
  return LTD_OK;
}

// Y = S^{-1} B (n columns of N_basis rows, ld nb_max) by conjugate gradients from
// Y = 0; convergence (every column's ||r|| <= tol ||b||) checked every 8 iterations.
ltd_status cg_solve(ltd_system *sys, int k, const double2 *B, int n, double2 *Y, int max_iter, double tol,
                    double *resid, int *iters, hipStream_t s) {
  const int nb = sys->kh[k].n_basis, ld = sys->nb_max;
  double2 *r = full_blk(sys, 5), *p = full_blk(sys, 6), *q = full_blk(sys, 7);
  double2 *sc = sys->at<double2>(sys->o_fscal);
  const int fc = std::min(1024, std::max(sys->max_cols, sys->n_states));
  double2 *rr = sc, *pq = sc + fc, *rrn = sc + 2 * fc, *b2 = sc + 3 * fc;
  LTD_HIP(launch_copy_rows(Y, ld, nullptr, 0, nb, n, true, s));
  LTD_HIP(launch_copy_rows(r, ld, B, ld, nb, n, false, s));
  LTD_HIP(launch_copy_rows(p, ld, B, ld, nb, n, false, s));
  LTD_HIP(launch_col_dots(r, r, nb, n, ld, rr, s));
  LTD_HIP(launch_col_dots(r, r, nb, n, ld, b2, s));
  std::vector<double2> hr(n), hb(n);
  double worst = 0.0;
  int it = 0;
  for (; it < max_iter;) {
    LTD_TRY(apply_s(sys, 0 <= k ? k : 0, p, ld, n, q, ld, s));
    LTD_HIP(launch_col_dots(p, q, nb, n, ld, pq, s));
    LTD_HIP(launch_cg_step(Y, r, p, q, rr, pq, nb, n, ld, s));
    LTD_HIP(launch_col_dots(r, r, nb, n, ld, rrn, s));
    ++it;
    if (it % 8 == 0 || it == max_iter) {
      LTD_HIP(hipMemcpyAsync(hr.data(), rrn, n * sizeof(double2), hipMemcpyDeviceToHost, s));
      LTD_HIP(hipMemcpyAsync(hb.data(), b2, n * sizeof(double2), hipMemcpyDeviceToHost, s));
      LTD_HIP(hipStreamSynchronize(s));
      worst = 0.0;
      for (int j = 0; j < n; ++j) worst = std::max(worst, hb[j].x > 0.0 ? std::sqrt(hr[j].x / hb[j].x) : 0.0);
      if (!std::isfinite(worst)) return LTD_ENONFINITE;
      if (worst <= tol) break;
    }
    LTD_HIP(launch_cg_dir(p, r, rr, rrn, nb, n, ld, s));
  }
  *resid = worst;
  *iters = it;
  return LTD_OK;
}

ltd_status read_status(ltd_system *sys, hipStream_t s, int *st) {
  LTD_HIP(hipStreamSynchronize(s));
  LTD_HIP(hipMemcpy(st, sys->ws + sys->o_status, sizeof(int), hipMemcpyDeviceToHost));
  return LTD_OK;
}

// Subspace matrices of a block X (N_basis x n): X^H T X, ..., made Hermitian, then
// S = L L^H, L^{-1}, and the S-orthonormal-basis T~, V~, P~, H~0 of the k-point's slots.
ltd_status setup_sub(ltd_system *sys, int k, const double2 *X, int ldx, hipStream_t s) {
  KHost &kh = sys->kh[k];
  const int n = sys->n_aux, nb = kh.n_basis;
  double2 *tv = sys->at<double2>(sys->o_tvps);  // 4 blocks N_basis x n, ld nb_max
  const int ldt = sys->nb_max;
  double2 *outs[4] = {tv, tv + (long long)ldt * n, tv + 2LL * ldt * n, tv + 3LL * ldt * n};
  const int lds[4] = {ldt, ldt, ldt, ldt};
  LTD_TRY(apply_cols(sys, k, FFT_MODE_TVPS, 0.0, X, ldx, n, outs, lds, s));
  // projection: X^H [TX | VX | PX | SX] -> n x 4n
  double2 *pr = sys->at<double2>(sys->o_proj);
  std::vector<ZProb> pp;
  for (int b = 0; b < 4; ++b) pp.push_back(zp(n, n, nb, X, ldx, outs[b], ldt, pr + (long long)b * n * n, n));
  LTD_TRY(gemm(sys, OP_C, OP_N, pp, s));
  double2 *subs = sys->at<double2>(kh.o_subs);
  LTD_HIP(launch_herm_split(pr, n, n, 4, subs, s));
  double2 *L = sys->at<double2>(kh.o_L), *Li = sys->at<double2>(kh.o_Linv);
  int *fail = sys->at<int>(sys->o_status) + 1;
  LTD_HIP(launch_cholesky(subs + 3LL * n * n, L, n, sys->at<int>(sys->o_status), fail, s));
  LTD_HIP(launch_trtri(L, Li, n, s));
  // tilde matrices: M~ = Li M Li^H for M in T, V, P
  double2 *tmp = sys->at<double2>(sys->o_tmp3);
  double2 *til = sys->at<double2>(kh.o_tilde);
  const long long n2 = (long long)n * n;
  const double2 one = make_double2(1.0, 0.0), zero = make_double2(0.0, 0.0);
  LTD_TRY(gemm1(sys, OP_N, OP_C, zp(n, n, n, subs, n, Li, n, tmp, n, one, zero, 3, n2, 0, n2), s));
  LTD_TRY(gemm1(sys, OP_N, OP_N, zp(n, n, n, Li, n, tmp, n, pr, n, one, zero, 3, 0, n2, n2), s));
  LTD_HIP(launch_herm_split(pr, n, n, 3, til, s));
  LTD_HIP(launch_axpby(til + 3 * n2, til, til + n2, 1.0, 1.0, n2, s));  // H~0 = T~ + V~_ref
  return LTD_OK;
}

ltd_status eig_bounds(ltd_system *sys, int k, hipStream_t s, double *lmin, double *lmax) {
  KHost &kh = sys->kh[k];
  const int n = sys->n_aux;
  const long long n2 = (long long)n * n;
  double2 *A = sys->at<double2>(sys->o_eigA);
  double *w = sys->at<double>(sys->o_eigw);
  LTD_HIP(hipMemcpyAsync(A, sys->at<double2>(kh.o_tilde) + 3 * n2, n2 * sizeof(double2), hipMemcpyDeviceToDevice, s));
  LTD_HIP(launch_jacobi(A, nullptr, w, n, s, sys->ws + sys->o_eigwork));
  std::vector<double> hw(n);
  LTD_HIP(hipStreamSynchronize(s));
  LTD_HIP(hipMemcpy(hw.data(), w, n * sizeof(double), hipMemcpyDeviceToHost));
  *lmin = hw[0];
  *lmax = hw[n - 1];
  return LTD_OK;
}

ltd_status upload_subdev(ltd_system *sys) {
  LTD_HIP(hipMemcpy(sys->ws + sys->o_subdev, sys->sd.data(), sys->sd.size() * sizeof(SubDev), hipMemcpyHostToDevice));
  return LTD_OK;
}

ltd_status prepare_dt(ltd_system *sys, double dt) {
  if (sys->cheb_dt == dt) return LTD_OK;
  std::vector<double2> c;
  for (int k = 0; k < sys->n_k; ++k) {
    if (!sys->kh[k].bound) continue;
    SubDev &d = sys->sd[k];
    const int deg = cheb_coef(d.r * dt, CHEB_KMAX, c);
    if (deg < 0) return LTD_EUNSUPPORTED;  // dt too large for the subspace spectrum
    d.K = std::max(deg, 1);
    for (int q = 0; q <= CHEB_KMAX; ++q) d.coef[q] = c[q];
    d.phase = make_double2(std::cos(dt * d.c0), -std::sin(dt * d.c0));
  }
  LTD_TRY(upload_subdev(sys));
  sys->cheb_dt = dt;
  return LTD_OK;
}

ltd_status build_step_tables(ltd_system *sys) {
  // K2 (muffin-tin rebuild) and the V~ projection GEMM over every bound k
  std::vector<ZProb> p1, p2, pv;
  const double2 *hx = sys->k2_step_h ? reinterpret_cast<const double2 *>(sys->k2_step_h) : sys->h;
  const int n = sys->n_aux;
  for (int k = 0; k < sys->n_k; ++k) {
    KHost &kh = sys->kh[k];
    if (!kh.bound) continue;
    double2 *ph = sys->at<double2>(kh.o_phit), *ye = sys->at<double2>(kh.o_yext);
    build_k2(sys, {hx}, ph + kh.n_g, kh.k_ext, {ye + kh.n_g}, kh.k_ext, n, p1, p2);
    // V~ = Phi~^H Y is Hermitian: block rows from the diagonal only
    for (int i0 = 0; i0 < n; i0 += PROJ_BLK)
      pv.push_back(zp(std::min(PROJ_BLK, n - i0), n - i0, kh.k_ext, ph + (long long)i0 * kh.k_ext, kh.k_ext,
                      ye + (long long)i0 * kh.k_ext, kh.k_ext, sys->at<double2>(kh.o_vstep) + i0 + (long long)i0 * n,
                      n));
  }
  const size_t cap = (size_t)4 * sys->n_atoms * sys->n_k * sizeof(ZProb) + 1024;
  // the rebuild's block products run beside the x/z transforms: unsplit, on few
  // CUs, with no reduction pass (a K split to fill the GPU took CUs from the
  // transforms and cost 7 us per pipelined step)
  LTD_TRY(upload_k2(sys, p1, p2, sys->k2_step, sys->o_k2_st1, sys->o_k2_st2, cap, 0));
  int tt = 0;
  gemm_plan(pv.data(), (int)pv.size(), &tt, sys->vproj_target, PART_TILES);
  sys->vstep_tab = pv;
  sys->vstep_tiles = tt;
  LTD_HIP(hipMemcpy(sys->ws + sys->o_vstep_tab, pv.data(), pv.size() * sizeof(ZProb), hipMemcpyHostToDevice));
  if (resid32(sys)) {  // the same two products on complex64 operands (ZProb pointers hold float2 data)
    std::vector<ZProb> p7, p6;
    const auto d2 = [](const void *p) { return reinterpret_cast<const double2 *>(p); };
    const float2 *dh = sys->at<float2>(sys->o_hstep32);
    for (int k = 0; k < sys->n_k; ++k) {
      KHost &kh = sys->kh[k];
      if (!kh.bound) continue;
      float2 *ph = sys->at<float2>(kh.o_phit32), *ye = sys->at<float2>(kh.o_yext32);
      for (int a = 0; a < sys->n_atoms; ++a) {
        const int sa = sys->n_mt[a] + sys->n_lo[a], r = kh.n_g + sys->mt_row32[a];
        p7.push_back(zp(sa, n, sa, d2(dh + sys->s_off[a]), sa, d2(ph + r), kh.k_ext,
                        reinterpret_cast<double2 *>(ye + r), kh.k_ext));
      }
      for (int i0 = 0; i0 < n; i0 += PROJ_BLK)
        p6.push_back(zp(std::min(PROJ_BLK, n - i0), n - i0, kh.k_ext, d2(ph + (long long)i0 * kh.k_ext), kh.k_ext,
                        d2(ye + (long long)i0 * kh.k_ext), kh.k_ext,
                        sys->at<double2>(kh.o_vstep) + i0 + (long long)i0 * n, n));
    }
    int t7 = 0, t6 = 0;
    gemm_plan(p7.data(), (int)p7.size(), &t7, 0, PART_TILES);  // unsplit: written in complex64 directly
    gemm_plan(p6.data(), (int)p6.size(), &t6, sys->vproj_target, PART_TILES);
    if (p7.size() * sizeof(ZProb) > (size_t)4 * sys->n_atoms * sys->n_k * sizeof(ZProb) + 1024) return LTD_EUNSUPPORTED;
    sys->k7_32 = p7;
    sys->k7_32_tiles = t7;
    sys->vstep32 = p6;
    sys->vstep32_tiles = t6;
    if (!p7.empty())
      LTD_HIP(hipMemcpy(sys->ws + sys->o_k7_32, p7.data(), p7.size() * sizeof(ZProb), hipMemcpyHostToDevice));
    LTD_HIP(hipMemcpy(sys->ws + sys->o_vstep32, p6.data(), p6.size() * sizeof(ZProb), hipMemcpyHostToDevice));
  }
  return LTD_OK;
}

StepCtx step_ctx(ltd_system *sys, const ltd_step_args *a) {
  StepCtx c{};
  c.sub = sys->at<SubDev>(sys->o_subdev);
  c.n_aux = sys->n_aux;
  c.n_states = sys->n_states;
  c.n_k = sys->n_k;
  c.h_in_lds = sys->h_in_lds ? 1 : 0;
  c.p_in_lds = sys->p_in_lds ? 1 : 0;
  c.rebuild = (a->mode == LTD_STEP_REBUILD) ? 1 : 0;
  c.resid = (c.rebuild && resid32(sys)) ? 1 : 0;
  c.step = a->step;
  c.step_rw = a->step;
  c.a_t = a->a_t;
  c.a_mid = a->a_mid;
  c.c_light = sys->c_light;
  c.occ = sys->occ;
  c.omega = sys->omega;
  c.dt = a->dt;
  c.theta = reinterpret_cast<double2 *>(a->theta);
  c.part = sys->at<double>(sys->o_part);
  c.taylor = a->taylor_order;
  c.nexc_out = a->nexc_out;
  c.status = sys->at<int>(sys->o_status);
  c.done = sys->at<int>(sys->o_status) + 8;  // zeroed at bind, reset by the step kernel's last block
  c.j_out = a->j_out;
  c.e_out = a->e_out;
  c.dmu_out = a->dmu_out;
  return c;
}

// Step stages (profiling tags): 0 Theta V(t), 1 x/z planes, 2 y lines, 3 muffin-tin
// blocks (K2), 4 projection of V~ (GEMM), 5 subspace step and observables, 6 map-back.
// Rebuild V~(t) of every k for the potential of this step (v_r_t, h_t).
// V~_step = Phi~_ext^H Y_ext of every bound k (one split-K GEMM table).
// parts: 1 the product (partials), 2 their reduction into V~, 3 both; the
// reduction only reads the partials, so repeating it gives the same V~.
ltd_status project_v(ltd_system *sys, hipStream_t s, int parts = 3) {
  if (resid32(sys)) {  // complex64 operands, FP32 matrix cores, FP64 sums across K tiles
    LTD_HIP(cgemm32_launch_table(OP_C, sys->at<ZProb>(sys->o_vstep32), sys->vstep32.data(), (int)sys->vstep32.size(),
                                 sys->vstep32_tiles, sys->at<double2>(sys->o_vpartials), s, parts, false));
    return LTD_OK;
  }
  LTD_HIP(gemm_launch_table(OP_C, OP_N, sys->at<ZProb>(sys->o_vstep_tab), sys->vstep_tab.data(),
                            (int)sys->vstep_tab.size(), sys->vstep_tiles, sys->at<double2>(sys->o_vpartials), 0, s,
                            parts));
  return LTD_OK;
}

// The step's muffin-tin blocks (the difference h(t) - h for the FP32 residual,
// in complex64) into the copy buffer the block products read, then the products.
// step: the device index of the step in a series (NULL: host_off or one set).
ltd_status step_blocks(ltd_system *sys, const ltd_step_args *a, const int *step, long long host_off, int n,
                       hipStream_t s) {
  if (resid32(sys)) {
    const double2 *src = a->h_t ? reinterpret_cast<const double2 *>(a->h_t) : sys->h;
    const bool series = a->h_t && a->h_stride;
    LTD_HIP(launch_copy_step32(sys->at<float2>(sys->o_hstep32), src, sys->blk_elems, series ? step : nullptr,
                               series ? a->h_stride : 0, series ? host_off : 0, sys->h, s));
    if (!sys->k7_32.empty())
      LTD_HIP(cgemm32_launch_table(OP_N, sys->at<ZProb>(sys->o_k7_32), sys->k7_32.data(), (int)sys->k7_32.size(),
                                   sys->k7_32_tiles, sys->at<double2>(sys->o_partials), s, 3, true));
    return LTD_OK;
  }
  if (a->h_t && a->h_stride)
    LTD_HIP(launch_copy_step(sys->at<double2>(sys->o_hstep), reinterpret_cast<const double2 *>(a->h_t),
                             sys->blk_elems, step, a->h_stride, host_off, nullptr, s));
  return run_k2(sys, sys->k2_step, n, s);
}

// Matrix-matrix route of the step's interstitial rows of Y_ext: the Fourier
// coefficients of Theta V(t) in the box of G differences, the dense block
// (Theta V(t))~(g - g') in the sphere-table order of Phi~_ext's rows, and
// Y_G = V^I(t) Phi~_G (GEMM), for every k-point.
ltd_status rebuild_v_mm(ltd_system *sys, const double *v, const int *step, long long stride, hipStream_t s,
                        Prof *pf) {
  const Grid g = grid_of(sys);
  const int n = sys->n_aux;
  double2 *box = sys->at<double2>(sys->o_box_step);
  LTD_HIP(mm_box_coefficients(g, sys->theta, v, step, stride, sys->at<double2>(sys->o_box_scr), box, s));
  LTD_MARK(pf, 0);
  std::vector<ZProb> py;
  for (int k = 0; k < sys->n_k; ++k) {
    const KHost &kh = sys->kh[k];
    double2 *vt = sys->at<double2>(kh.o_mmVt);
    LTD_HIP(mm_dense(2, g, sys->at<int>(kh.o_gint), sys->at<double>(kh.o_gk), sys->at<int>(kh.o_ptsg), kh.n_g,
                     nullptr, box, vt, kh.n_g, s));
    py.push_back(zp(kh.n_g, n, kh.n_g, vt, kh.n_g, sys->at<double2>(kh.o_phit), kh.k_ext,
                    sys->at<double2>(kh.o_yext), kh.k_ext));
  }
  LTD_MARK(pf, 1);
  LTD_TRY(gemm(sys, OP_N, OP_N, py, s));
  LTD_MARK(pf, 2);
  return LTD_OK;
}

// host_step >= 0: the step index is known on the host (adjoint); otherwise the
// series are indexed by the device step counter.
ltd_status rebuild_v(ltd_system *sys, const ltd_step_args *a, hipStream_t s, Prof *pf = nullptr,
                     int host_step = -1) {
  const Grid g = rgrid_of(sys);
  const int n = sys->n_aux;
  const void *hx = k2_source(sys, a);
  if (hx != sys->k2_step_h) {  // host tables before any launch of the step
    sys->k2_step_h = hx;
    LTD_TRY(build_step_tables(sys));
  }
  // muffin-tin branch (blocks of the step, K2 into the Y rows past the G block)
  // on the side stream, beside the FFT chain; serial when stages are timed
  const bool fork = pf == nullptr && sys->side != nullptr;
  hipStream_t sb = s;
  if (fork) {
    LTD_HIP(hipEventRecord(sys->ev_fork, s));
    LTD_HIP(hipStreamWaitEvent(sys->side, sys->ev_fork, 0));
    sb = sys->side;
  }
  const bool r32 = resid32(sys);
  const int *hstep = host_step >= 0 ? nullptr : a->step;
  const long long hoff = host_step >= 0 ? (long long)host_step * a->h_stride : 0;
  if (fork) {
    LTD_TRY(step_blocks(sys, a, hstep, hoff, n, sb));
    LTD_HIP(hipEventRecord(sys->ev_join, sb));
  }
  if (sys->route == LTD_ROUTE_MM) {  // interstitial V_sub(t) by the dense block of the step's potential
    const double *v = a->v_r_t ? a->v_r_t : sys->v_r;
    const int *dstep = nullptr;
    if (a->v_r_t && a->v_stride) {
      if (host_step >= 0) v += (long long)host_step * a->v_stride;
      else dstep = a->step;
    }
    LTD_TRY(rebuild_v_mm(sys, v, dstep, a->v_stride, s, pf));
  } else {
  const void *thv = r32 ? static_cast<const void *>(sys->at<float>(sys->o_zero32))
                        : static_cast<const void *>(sys->at<double>(sys->o_thv_rb));
  if (a->v_r_t) {
    const double *v = a->v_r_t;
    const int *dstep = nullptr;
    if (a->v_stride) {
      if (host_step >= 0) v += (long long)host_step * a->v_stride;
      else dstep = a->step;
    }
    LTD_TRY(rebuild_potential(sys, v, dstep, a->v_stride, sys->at<double>(sys->o_thv_step), r32, s));
    thv = sys->at<double>(sys->o_thv_step);
  }
  LTD_MARK(pf, 0);
  const long long slab = (long long)fft_rb_slab_values(g) * n;
  for (int k0 = 0; k0 < sys->n_k; k0 += FFT_MAXK) {
    const int nk = std::min(FFT_MAXK, sys->n_k - k0);
    FftKArgs ka{};
    for (int i = 0; i < nk; ++i) {
      const KHost &kh = sys->kh[k0 + i];
      ka.sph[i] = sphere_of(sys, k0 + i);
      ka.slab_in[i] = sys->at<double2>(kh.o_cache);
      ka.slab_out[i] = reinterpret_cast<double2 *>(sys->ws + sys->o_stepslab + (size_t)i * slab * rb_elem(sys));
      ka.out[i].o0 = sys->at<double2>(kh.o_yext);
      ka.out[i].o0f = r32 ? sys->at<float2>(kh.o_yext32) : nullptr;
      ka.out[i].ld0 = kh.k_ext;
    }
    // x/z transforms and the Theta V product per y plane, then y transforms per kz plane;
    // timed stages launch the x/z kernel PROF_XZ_REPS times back to back (it reads
    // the cache and Theta V and writes the slab: the same slab every time)
    for (int r = 0; r < (pf ? PROF_XZ_REPS : 1); ++r)
      LTD_HIP(fft_rb_step(g, ka, nk, n, thv, s, 0, r32, sys->rb_variant));
    LTD_MARK(pf, 1);
    for (int i = 0; i < nk; ++i) ka.slab_in[i] = ka.slab_out[i];
    LTD_HIP(fft_rb_step(g, ka, nk, n, thv, s, 1, r32, 0));
    LTD_MARK(pf, 2);
  }
  }
  if (fork) LTD_HIP(hipStreamWaitEvent(s, sys->ev_join, 0));
  else LTD_TRY(step_blocks(sys, a, hstep, hoff, n, s));
  LTD_MARK(pf, 3);
  LTD_TRY(project_v(sys, s));
  LTD_MARK(pf, 4);
  return LTD_OK;
}

// Rebuild of Y_ext within a pipelined step; the projection product follows on
// s.  After the first x/z launch the call enqueues the current step's work on
// side2 (the reduction of the previous product's partials into V~ once s has
// passed ev_p0, the assembly of H~(mid), recorded as ev_asm, and the
// exponential of exp_ctx); the y transforms wait for ev_asm, so the product
// that rewrites the partials comes after the assembly.  The muffin-tin branch
// advances its own step index rk on the side stream before it reads the blocks
// of the step.  When the call hands in a potential, Theta V alternates between
// two buffers: step i of a capture of kc steps reads buffer i mod 2, which holds
// it already, and the synthesis of the next step's (its own step index rv, on
// side3) writes the other one, beside the x/z transforms, and joins s with the
// muffin-tin rows and the assembly before the y transforms, so that the next
// x/z launch waits on no other stream.  The last step of a capture writes
// buffer 0, where the next capture (or the prologue of ltd_propagate) starts;
// when that step reads buffer 0 itself (kc odd) the synthesis waits for its x/z
// transforms and the capture's end joins it.
ltd_status rebuild_v_pipe(ltd_system *sys, const ltd_step_args *a, hipStream_t s, int i_cap, int kc,
                          const StepCtx &exp_ctx) {
  const Grid g = rgrid_of(sys);
  const int n = sys->n_aux;
  int *rk = sys->at<int>(sys->o_status) + 12, *rv = rk + 2;
  const void *hx = k2_source(sys, a);
  if (hx != sys->k2_step_h) {
    sys->k2_step_h = hx;
    LTD_TRY(build_step_tables(sys));
  }
  const bool r32 = resid32(sys);
  // the side streams' work of the step depends on s only up to here; it is
  // captured after the first x/z launch, so that the x/z kernel is the first
  // node its predecessor releases
  LTD_HIP(hipEventRecord(sys->ev_fork, s));
  const void *thv = r32 ? static_cast<const void *>(sys->at<float>(sys->o_zero32))
                        : static_cast<const void *>(sys->at<double>(sys->o_thv_rb));
  double *const tbuf[2] = {sys->at<double>(sys->o_thv_step), sys->at<double>(sys->o_thv_step2)};
  const bool last = i_cap == kc - 1;
  double *const tnext = last ? tbuf[0] : tbuf[(i_cap + 1) & 1];
  const bool early = a->v_r_t && tnext != tbuf[i_cap & 1];  // the next Theta V beside the x/z transforms
  if (a->v_r_t) thv = tbuf[i_cap & 1];
  const long long slab = (long long)fft_rb_slab_values(g) * n;
  for (int k0 = 0; k0 < sys->n_k; k0 += FFT_MAXK) {
    const int nk = std::min(FFT_MAXK, sys->n_k - k0);
    FftKArgs ka{};
    for (int i = 0; i < nk; ++i) {
      const KHost &kh = sys->kh[k0 + i];
      ka.sph[i] = sphere_of(sys, k0 + i);
      ka.slab_in[i] = sys->at<double2>(kh.o_cache);
      ka.slab_out[i] = reinterpret_cast<double2 *>(sys->ws + sys->o_stepslab + (size_t)i * slab * rb_elem(sys));
      ka.out[i].o0 = sys->at<double2>(kh.o_yext);
      ka.out[i].o0f = r32 ? sys->at<float2>(kh.o_yext32) : nullptr;
      ka.out[i].ld0 = kh.k_ext;
    }
    LTD_HIP(fft_rb_step(g, ka, nk, n, thv, s, 0, r32, sys->rb_variant));
    if (k0 == 0) {  // the muffin-tin rows on side, the exponential of the current step on side2
      LTD_HIP(hipStreamWaitEvent(sys->side, sys->ev_fork, 0));
      LTD_HIP(launch_lookahead(rk, sys->side));
      LTD_TRY(step_blocks(sys, a, rk, 0, n, sys->side));
      LTD_HIP(hipEventRecord(sys->ev_join, sys->side));
      LTD_HIP(hipStreamWaitEvent(sys->side2, sys->ev_p0, 0));
      LTD_TRY(project_v(sys, sys->side2, 2));
      LTD_HIP(launch_assemble(exp_ctx, sys->side2));
      if (a->theta_hist)  // the states before the step, for a checkpointed backward pass
        LTD_HIP(launch_record_theta(exp_ctx, reinterpret_cast<double2 *>(a->theta_hist), a->hist_len, sys->side2));
      LTD_HIP(hipEventRecord(sys->ev_asm, sys->side2));
      LTD_HIP(launch_step_only(exp_ctx, sys->side2, true));
      if (early) {  // after ev_fork: the x/z launch of step i - 1 has read tnext
        LTD_HIP(hipStreamWaitEvent(sys->side3, sys->ev_fork, 0));
        LTD_HIP(launch_lookahead(rv, sys->side3));
        LTD_TRY(rebuild_potential(sys, a->v_r_t, a->v_stride ? rv : nullptr, a->v_stride, tnext, r32, sys->side3));
        LTD_HIP(hipEventRecord(sys->ev_syn, sys->side3));
      }
    }
    if (a->v_r_t && !early && k0 + FFT_MAXK >= sys->n_k) {  // Theta V read: the next step's synthesis
      LTD_HIP(hipEventRecord(sys->ev_xz, s));
      LTD_HIP(hipStreamWaitEvent(sys->side3, sys->ev_xz, 0));
      LTD_HIP(launch_lookahead(rv, sys->side3));
      LTD_TRY(rebuild_potential(sys, a->v_r_t, a->v_stride ? rv : nullptr, a->v_stride, tnext, r32, sys->side3));
      LTD_HIP(hipEventRecord(sys->ev_syn, sys->side3));
    }
    for (int i = 0; i < nk; ++i) ka.slab_in[i] = ka.slab_out[i];
    // the waits for the muffin-tin rows and the assembly that reads V~ go before
    // the y transforms, not before the projection: both are done by then, and
    // the projection keeps the y transforms as its only dependency (measured:
    // 14 us per step less in the replayed graph)
    LTD_HIP(hipStreamWaitEvent(s, sys->ev_join, 0));
    LTD_HIP(hipStreamWaitEvent(s, sys->ev_asm, 0));
    if (early) LTD_HIP(hipStreamWaitEvent(s, sys->ev_syn, 0));
    LTD_HIP(fft_rb_step(g, ka, nk, n, thv, s, 1, r32, 0));
  }
  return LTD_OK;
}

ltd_status map_back(ltd_system *sys, const ltd_step_args *a, hipStream_t s) {
  if (!a->c_out) return LTD_OK;
  std::vector<ZProb> pp;
  long long coff = 0;
  const int n = sys->n_aux, ns = sys->n_states;
  for (int k = 0; k < sys->n_k; ++k) {
    const KHost &kh = sys->kh[k];
    pp.push_back(zp(kh.n_basis, ns, n, kh.phi, kh.ldphi, reinterpret_cast<double2 *>(a->theta) + (long long)k * n * ns,
                    n, reinterpret_cast<double2 *>(a->c_out) + coff, kh.n_basis));
    coff += (long long)kh.n_basis * ns;
  }
  return gemm(sys, OP_N, OP_N, pp, s);
}

ltd_status check_step_args(ltd_system *sys, const ltd_step_args *a) {
  if (!sys || !a) return LTD_EINVAL;
  if (!sys->ws) return LTD_ESTATE;
  for (int k = 0; k < sys->n_k; ++k)
    if (!sys->kh[k].bound) return LTD_ESTATE;
  if (a->mode != LTD_STEP_REBUILD && a->mode != LTD_STEP_AFFINE) return LTD_EINVAL;
  if (!(std::isfinite(a->dt)) || a->dt == 0.0) return LTD_EINVAL;
  if (!a->a_t || !a->a_mid || !a->step || !a->theta || !a->j_out || !a->e_out || !a->dmu_out) return LTD_EINVAL;
  if (!aligned16(a->theta) || (a->c_out && !aligned16(a->c_out))) return LTD_EALIGN;
  if (a->h_t && !aligned16(a->h_t)) return LTD_EALIGN;
  if (a->v_stride < 0 || a->h_stride < 0) return LTD_EINVAL;
  if (a->v_stride && a->v_stride < sys->ngrid) return LTD_ESHAPE;
  if (a->h_stride && a->h_stride < sys->blk_elems) return LTD_ESHAPE;
  if (a->taylor_order < 0 || a->taylor_order > TAYLOR_MAX) return LTD_EINVAL;
  if (a->theta_hist && (a->hist_len < 1 || !aligned16(a->theta_hist))) return a->hist_len < 1 ? LTD_ESHAPE : LTD_EALIGN;
  if (a->taylor_order > 0)  // the explicit step diverges beyond the critical time step (Eq. (20))
    for (int k = 0; k < sys->n_k; ++k)
      if (std::fabs(a->dt) > 0.2 / (sys->kh[k].lam_max - sys->kh[k].lam_min)) return LTD_ESTEP;
  return LTD_OK;
}

void drop_graphs(ltd_system *sys) {
  for (int t = 0; t < GRAPH_TIERS; ++t) {
    if (sys->gexec[t]) (void)hipGraphExecDestroy(sys->gexec[t]);
    if (sys->graph[t]) (void)hipGraphDestroy(sys->graph[t]);
    sys->gexec[t] = nullptr;
    sys->graph[t] = nullptr;
  }
}

// Pipelined steps (REBUILD): each step rebuilds V~ of the next step on `s`
// while the exponential of the current step runs on side2.  The rebuild's step
// indices are counters of their own (set at the start of a propagate call, then
// advanced by one per step and clamped to the call's last step), so the rebuild
// chain never waits for the exponential; side2 waits for the V~ it assembles
// (ev_p0), and the projection that overwrites V~ waits until it was assembled
// (ev_asm).  The projection's split-K reduction into V~ runs on side2 at the
// start of the next step, before the assembly that reads V~ (the partials of
// the last product of a call are reduced once more after its graphs; the
// first step of a call reduces the prologue's partials a second time, which
// gives the same V~).  `first`: the first step of a capture (Theta V of its
// rebuild was made before the capture); `join`: the last step joins side2 and
// side3 back into s.  map_back is a no-op without C.
ltd_status pipelined_step(ltd_system *sys, const ltd_step_args *a, hipStream_t s, int i_cap, int kc) {
  const bool join = i_cap == kc - 1;
  const StepCtx c = step_ctx(sys, a);
  // side2's work (reduction, assembly, exponential) depends on s only up to
  // here (ev_p0); it is captured after the first x/z launch, which leaves the
  // graph's dependencies as they are but puts the x/z kernel first in its
  // launch order (measured: 2.7 us per step less)
  LTD_HIP(hipEventRecord(sys->ev_p0, s));
  LTD_TRY(rebuild_v_pipe(sys, a, s, i_cap, kc, c));
  LTD_TRY(project_v(sys, s, 1));
  // the map-back GEMM shares the split-K partials with the rebuild's GEMMs: it
  // runs on s, after the step (a join every step when C is requested)
  if (join || a->c_out) {
    LTD_HIP(hipEventRecord(sys->ev_pj, sys->side2));
    LTD_HIP(hipStreamWaitEvent(s, sys->ev_pj, 0));
  }
  if (join && a->v_r_t) LTD_HIP(hipStreamWaitEvent(s, sys->ev_syn, 0));
  LTD_TRY(map_back(sys, a, s));
  return LTD_OK;
}

ltd_status step_once(ltd_system *sys, const ltd_step_args *a, hipStream_t s, Prof *pf = nullptr) {
  if (a->mode == LTD_STEP_REBUILD) LTD_TRY(rebuild_v(sys, a, s, pf));
  if (a->theta_hist)
    LTD_HIP(launch_record_theta(step_ctx(sys, a), reinterpret_cast<double2 *>(a->theta_hist), a->hist_len, s));
  LTD_HIP(launch_step(step_ctx(sys, a), s));
  LTD_MARK(pf, 5);
  LTD_TRY(map_back(sys, a, s));
  LTD_MARK(pf, 6);
  return LTD_OK;
}

// Fork/join ledger of a capture, taken before it ends: every side stream that
// joined the capture (it waited on an event of the capture stream's chain) must
// have its last captured work among the ancestors of the capture stream's
// current tail, i.e. joined back; otherwise LTD_ECAPTURE (the capture code left
// work dangling, which the runtime would report, or mishandle, at the end).
ltd_status check_joined(ltd_system *sys) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  unsigned long long id0 = 0;
  const hipGraphNode_t *d0 = nullptr;
  size_t n0 = 0;
  LTD_HIP(hipStreamGetCaptureInfo_v2(sys->cap_stream, &cs, &id0, nullptr, &d0, &n0));
  if (cs != hipStreamCaptureStatusActive) return LTD_ECAPTURE;
  std::unordered_set<hipGraphNode_t> anc;
  std::vector<hipGraphNode_t> todo(d0, d0 + n0), deps;
  while (!todo.empty()) {
    const hipGraphNode_t node = todo.back();
    todo.pop_back();
    if (!anc.insert(node).second) continue;
    size_t nd = 0;
    LTD_HIP(hipGraphNodeGetDependencies(node, nullptr, &nd));
    if (nd == 0) continue;
    deps.assign(nd, nullptr);
    LTD_HIP(hipGraphNodeGetDependencies(node, deps.data(), &nd));
    todo.insert(todo.end(), deps.begin(), deps.begin() + nd);
  }
  for (hipStream_t x : {sys->side, sys->side2, sys->side3}) {
    if (!x) continue;
    hipStreamCaptureStatus xs = hipStreamCaptureStatusNone;
    unsigned long long id = 0;
    const hipGraphNode_t *d = nullptr;
    size_t nd = 0;
    LTD_HIP(hipStreamGetCaptureInfo_v2(x, &xs, &id, nullptr, &d, &nd));
    if (xs != hipStreamCaptureStatusActive || id != id0) continue;  // not forked in this capture
    for (size_t i = 0; i < nd; ++i)
      if (!anc.count(d[i])) return LTD_ECAPTURE;
  }
  return LTD_OK;
}

// k steps in one capture (a replay boundary per k steps); the graph is kept
ltd_status capture_steps(ltd_system *sys, const ltd_step_args *a, int k, bool pipe, hipGraph_t *g,
                         hipGraphExec_t *x) {
  if (*x) return LTD_OK;
  if (!sys->cap_stream) LTD_HIP(hipStreamCreateWithFlags(&sys->cap_stream, hipStreamNonBlocking));
  LTD_HIP(hipStreamBeginCapture(sys->cap_stream, hipStreamCaptureModeThreadLocal));
  ltd_status st = LTD_OK;
  for (int i = 0; i < k && st == LTD_OK; ++i)
    st = pipe ? pipelined_step(sys, a, sys->cap_stream, i, k) : step_once(sys, a, sys->cap_stream);
  if (st == LTD_OK) st = check_joined(sys);
  hipGraph_t gr = nullptr;
  const hipError_t ec = hipStreamEndCapture(sys->cap_stream, &gr);
  if (st != LTD_OK) {
    if (gr) (void)hipGraphDestroy(gr);
    return st;
  }
  if (ec != hipSuccess) return LTD_EHIP;
  *g = gr;
  LTD_HIP(hipGraphInstantiate(x, gr, nullptr, nullptr, 0));
  return LTD_OK;
}

// The graphs of every tier a call of n_steps with these arguments replays
// (captured now if they are not kept from an earlier call with the same ones).
ltd_status ensure_graphs(ltd_system *sys, const ltd_step_args *a, int n_steps, bool pipe) {
  const bool same = sys->gvalid && sys->gpipe == pipe && std::memcmp(&sys->gargs, a, sizeof(ltd_step_args)) == 0;
  if (!same) {
    drop_graphs(sys);
    sys->gargs = *a;
    sys->gpipe = pipe;
    sys->gvalid = true;
  }
  int left = n_steps;
  for (int t = 0; t < GRAPH_TIERS; ++t) {
    const int reps = left / GRAPH_STEPS[t];
    if (reps == 0) continue;
    LTD_TRY(capture_steps(sys, a, GRAPH_STEPS[t], pipe, &sys->graph[t], &sys->gexec[t]));
    left -= reps * GRAPH_STEPS[t];
  }
  return LTD_OK;
}

// the step tables a rebuild reads must be current before a capture
ltd_status refresh_step_tables(ltd_system *sys, const ltd_step_args *a) {
  if (a->mode == LTD_STEP_REBUILD && k2_source(sys, a) != sys->k2_step_h) {
    sys->k2_step_h = k2_source(sys, a);
    LTD_TRY(build_step_tables(sys));
  }
  return LTD_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char *ltd_status_string(ltd_status st) {
  switch (st) {
    case LTD_OK: return "ok";
    case LTD_EINVAL: return "invalid argument";
    case LTD_ESHAPE: return "inconsistent sizes or leading dimensions";
    case LTD_EALIGN: return "complex pointer not 16-byte aligned";
    case LTD_ESTATE: return "call out of order (workspace or subspace not bound)";
    case LTD_EWORKSPACE: return "workspace too small";
    case LTD_EUNSUPPORTED: return "size or mode not supported by this build";
    case LTD_EHIP: return "HIP runtime error";
    case LTD_ENOTSPD: return "subspace overlap not positive definite";
    case LTD_ENONFINITE: return "non-finite current or energy";
    case LTD_ESPECTRUM: return "subspace spectrum left the propagator interval";
    case LTD_ESTEP: return "time step above the critical time step of the explicit propagator";
    case LTD_ECAPTURE: return "graph capture: a forked stream was not joined back";
    default: return "unknown status";
  }
}

ltd_status ltd_create(const ltd_system_desc *d, int precision, size_t *ws_bytes, ltd_system **out) {
  if (!d || !ws_bytes || !out) return LTD_EINVAL;
  *out = nullptr;
  if (precision != LTD_FP64 && precision != LTD_FP32_RESID) return LTD_EUNSUPPORTED;
  if (d->n_k < 1 || d->n_atoms < 0 || d->n_aux < 1 || d->n_states < 1 || d->n_states > d->n_aux ||
      d->max_cols < 1)
    return LTD_ESHAPE;
  if (!d->n_g || !d->g_int || !d->gk_cart || !d->theta_r || !d->v_r || !d->amat || !d->k_weight) return LTD_EINVAL;
  if (d->n_atoms > 0 && (!d->n_mt || !d->n_lo || !d->h || !d->o || !d->pz)) return LTD_EINVAL;
  if (!(d->omega > 0.0) || !(d->c_light > 0.0) || !std::isfinite(d->occ)) return LTD_EINVAL;
  if (!aligned16(d->amat) || (d->n_atoms > 0 && (!aligned16(d->h) || !aligned16(d->o) || !aligned16(d->pz))))
    return LTD_EALIGN;
  if (d->n_aux > 320) return LTD_EUNSUPPORTED;
  if (d->interstitial_route != LTD_ROUTE_FFT && d->interstitial_route != LTD_ROUTE_MM &&
      d->interstitial_route != LTD_ROUTE_FFT_PLANES)
    return LTD_EINVAL;
  if (d->interstitial_route == LTD_ROUTE_MM && precision != LTD_FP64) return LTD_EUNSUPPORTED;
  auto *sys = new ltd_system();
  sys->n_k = d->n_k;
  sys->n1 = d->grid[0];
  sys->n2 = d->grid[1];
  sys->n3 = d->grid[2];
  sys->ngrid = (long long)sys->n1 * sys->n2 * sys->n3;
  Grid &g = sys->grid;
  g.n1 = sys->n1;
  g.n2 = sys->n2;
  g.n3 = sys->n3;
  if (!fft_plan_length(g.n1, &g.p1) || !fft_plan_length(g.n2, &g.p2) || !fft_plan_length(g.n3, &g.p3)) {
    delete sys;
    return LTD_EUNSUPPORTED;
  }
  sys->theta = d->theta_r;
  sys->v_r = d->v_r;
  sys->n_atoms = d->n_atoms;
  int ao = 0, lo = 0;
  long long so = 0;
  for (int a = 0; a < d->n_atoms; ++a) {
    if (d->n_mt[a] < 1 || d->n_lo[a] < 0) {
      delete sys;
      return LTD_ESHAPE;
    }
    sys->n_mt.push_back(d->n_mt[a]);
    sys->n_lo.push_back(d->n_lo[a]);
    sys->a_off.push_back(ao);
    sys->l_off.push_back(lo);
    sys->s_off.push_back((int)so);
    const int s = d->n_mt[a] + d->n_lo[a];
    ao += d->n_mt[a];
    lo += d->n_lo[a];
    so += (long long)s * s;
  }
  sys->n_a = ao;
  sys->n_lo_tot = lo;
  sys->n_loc = ao + lo;
  sys->blk_elems = so;
  sys->amat = reinterpret_cast<const double2 *>(d->amat);
  sys->h = reinterpret_cast<const double2 *>(d->h);
  sys->o = reinterpret_cast<const double2 *>(d->o);
  sys->pz = reinterpret_cast<const double2 *>(d->pz);
  sys->omega = d->omega;
  sys->c_light = d->c_light;
  sys->occ = d->occ;
  sys->n_aux = d->n_aux;
  sys->n_states = d->n_states;
  sys->max_cols = d->max_cols;
  sys->precision = precision;
  sys->route = d->interstitial_route == LTD_ROUTE_MM ? LTD_ROUTE_MM : LTD_ROUTE_FFT;
  sys->planes_only = d->interstitial_route == LTD_ROUTE_FFT_PLANES;
  // G sets, box, sphere tables
  long long gtot = 0;
  int bx = 0, by = 0, bz = 0;
  for (int k = 0; k < d->n_k; ++k) {
    if (d->n_g[k] < 1) {
      delete sys;
      return LTD_ESHAPE;
    }
    gtot += d->n_g[k];
  }
  sys->g_int.assign(d->g_int, d->g_int + 3 * gtot);
  sys->gk.assign(d->gk_cart, d->gk_cart + 3 * gtot);
  for (long long i = 0; i < gtot; ++i) {
    bx = std::max(bx, std::abs(sys->g_int[3 * i]));
    by = std::max(by, std::abs(sys->g_int[3 * i + 1]));
    bz = std::max(bz, std::abs(sys->g_int[3 * i + 2]));
  }
  if (2 * bx >= g.n1 || 2 * by >= g.n2 || 2 * bz >= g.n3) {
    delete sys;
    return LTD_ESHAPE;
  }
  g.bx = bx;
  g.by = by;
  g.bz = bz;
  g.nbx = 2 * bx + 1;
  g.nby = 2 * by + 1;
  g.nbz = 2 * bz + 1;
  g.d1 = g.n1;
  g.d2 = g.n2;
  {
    Grid r = g;
    r.n1 = fft_rb_length(g.n1, bx);
    r.n2 = fft_rb_length(g.n2, by);
    r.n3 = fft_rb_length(g.n3, bz);
    const bool smaller = r.n1 != g.n1 || r.n2 != g.n2 || r.n3 != g.n3;
    if (smaller && fft_rb_fast(r) && fft_plan_length(r.n1, &r.p1) && fft_plan_length(r.n2, &r.p2) &&
        fft_plan_length(r.n3, &r.p3)) {
      sys->rgrid = r;
      sys->rb_synth = true;
    } else {
      sys->rgrid = g;
    }
    // the FP32 residual runs on the register transforms only
    if (precision == LTD_FP32_RESID && !fft_rb_fast(sys->rgrid)) {
      delete sys;
      return LTD_EUNSUPPORTED;
    }
    sys->ap_red = sys->rb_synth && sys->route == LTD_ROUTE_FFT;
  }
  if (fft_plane_lds_bytes(g) > 160 * 1024 || fft_line_lds_bytes(g) > 160 * 1024) {
    delete sys;
    return LTD_EUNSUPPORTED;
  }
  long long goff = 0;
  size_t aoff = 0;
  sys->nb_max = 0;
  for (int k = 0; k < d->n_k; ++k) {
    KHost kh{};
    kh.n_g = d->n_g[k];
    kh.n_basis = kh.n_g + sys->n_lo_tot;
    kh.k_ext = kh.n_g + sys->n_loc;
    kh.g_off = goff;
    kh.amat_off = aoff;
    sys->nb_max = std::max(sys->nb_max, kh.n_basis);
    // CSR of sphere points by kz plane; injectivity of g mod N
    std::vector<std::vector<int>> byplane(g.nbz);
    std::vector<char> seen((size_t)g.n1 * g.n2 * g.n3, 0);
    for (int i = 0; i < kh.n_g; ++i) {
      const int *gi = &sys->g_int[3 * (goff + i)];
      const int x = (gi[0] % g.n1 + g.n1) % g.n1, y = (gi[1] % g.n2 + g.n2) % g.n2, z = (gi[2] % g.n3 + g.n3) % g.n3;
      const size_t lin = (size_t)x + (size_t)g.n1 * (y + (size_t)g.n2 * z);
      if (seen[lin]) {
        delete sys;
        return LTD_ESHAPE;
      }
      seen[lin] = 1;
      byplane[gi[2] + bz].push_back(i);
    }
    kh.plane_ptr.push_back(0);
    for (int p = 0; p < g.nbz; ++p) {
      int xlo = g.nbx, xhi = 0;  // box-x lines of the plane's points
      for (int i : byplane[p]) {
        xlo = std::min(xlo, sys->g_int[3 * (goff + i)] + g.bx);
        xhi = std::max(xhi, sys->g_int[3 * (goff + i)] + g.bx + 1);
      }
      kh.plane_x.push_back(xlo < xhi ? xlo : 0);
      kh.plane_x.push_back(xlo < xhi ? xhi : 0);
      for (int i : byplane[p]) {
        const int *gi = &sys->g_int[3 * (goff + i)];
        const int x = (gi[0] % g.n1 + g.n1) % g.n1, y = (gi[1] % g.n2 + g.n2) % g.n2;
        kh.pts_g.push_back(i);
        kh.pts_xy.push_back(y * g.n1 + x);
        if (sys->ap_red) {
          const int rn1 = sys->rgrid.n1, rn2 = sys->rgrid.n2;
          const int xa = (gi[0] % rn1 + rn1) % rn1, ya = (gi[1] % rn2 + rn2) % rn2;
          kh.pts_xy_a.push_back(ya * rn1 + xa);
        }
      }
      kh.plane_ptr.push_back((int)kh.pts_g.size());
    }
    sys->kh.push_back(kh);
    goff += kh.n_g;
    aoff += (size_t)sys->n_a * kh.n_g;
    sys->kw.push_back(d->k_weight[k]);
  }
  // columns per apply pass: FFT slabs (4 in + 5 out fields) within ~6 GB; when
  // the columns take several passes, a multiple of the GEMMs' 64-column tile
  // (a 45-column pass computes 64 columns' worth of muffin-tin MFMA work)
  const Grid &ag = sys->ap_red ? sys->rgrid : g;  // grid of the apply's FFT passes
  // the box route runs where the apply grid has the register plane and x/z kernels
  // (on the rebuild grid, or the grid itself when it is the rebuild grid); its
  // slabs hold box arrays: 4 y images (or the 5 sphere-order fields) in, 5 out
  // (the passes keep the plane route's width: one pass of 300 heterostructure
  // columns made the muffin-tin GEMMs slower, 3.55 -> 4.33 ms, and the step too)
  sys->ap_box = sys->route == LTD_ROUTE_FFT && !sys->planes_only && (sys->ap_red || !sys->rb_synth) &&
                fft_ap_box_ok(ag);
  const long long per_col = 9LL * ag.nbz * ag.n1 * ag.n2 * (long long)sizeof(double2);
  const int cmax = std::max(sys->max_cols, sys->n_aux);
  sys->chunk = (int)std::max(1LL, std::min<long long>(cmax, (6LL << 30) / per_col));
  if (sys->chunk < cmax && sys->chunk >= 64) sys->chunk -= sys->chunk % 64;
  const int n = sys->n_aux;
  const long long n2 = (long long)n * n;
  sys->h_in_lds = step_lds_bytes(n, true, true) <= 150 * 1024;
  sys->p_in_lds = sys->h_in_lds && step_lds_bytes(n, true, false, true) <= 150 * 1024;
  // workspace plan
  Arena ar;
  sys->o_tw1 = ar.take(g.n1 * sizeof(double2));
  sys->o_tw2 = ar.take(g.n2 * sizeof(double2));
  sys->o_tw3 = ar.take(g.n3 * sizeof(double2));
  sys->o_thv = ar.take(sys->ngrid * sizeof(double));
  sys->o_thv_rb = ar.take(sys->ngrid * sizeof(double));
  sys->o_thv_step = ar.take(sys->ngrid * sizeof(double));
  sys->o_thv_step2 = ar.take(sys->ngrid * sizeof(double));
  if (sys->ap_red) {
    const size_t rn = (size_t)sys->rgrid.n1 * sys->rgrid.n2 * sys->rgrid.n3;
    sys->o_th_ap = ar.take(rn * sizeof(double));
    sys->o_thv_ap = ar.take(rn * sizeof(double));
  }
  if (sys->ap_red || sys->ap_box) sys->o_ones = ar.take(sys->ngrid * sizeof(double));
  if (sys->ap_box) {
    const size_t rn = (size_t)ag.n1 * ag.n2 * ag.n3;
    sys->o_th_x = ar.take(rn * sizeof(double));
    sys->o_thv_x = sys->ap_red ? ar.take(rn * sizeof(double)) : 0;  // else the rebuild's Theta V
  }
  // [0..1] status, [8] step-kernel block counter, [12..13] and [14..15] step index
  // and last step of the pipelined rebuild (muffin-tin branch, potential synthesis)
  sys->o_status = ar.take(64);
  sys->o_part = ar.take((size_t)PART_STRIDE * sys->n_k * sys->n_states * sizeof(double));
  sys->o_partials = ar.take((size_t)PART_TILES * 64 * 64 * sizeof(double2));
  sys->o_vpartials = ar.take((size_t)PART_TILES * 64 * 64 * sizeof(double2));
  const bool mm = sys->route == LTD_ROUTE_MM;
  const long long slab_f = mm ? 0 : (long long)ag.nbz * ag.n1 * ag.n2 * sys->chunk;
  sys->o_slab_in = ar.take(4 * slab_f * sizeof(double2));
  sys->o_slab_out = ar.take(5 * slab_f * sizeof(double2));
  sys->o_W = ar.take((size_t)sys->n_loc * sys->chunk * sizeof(double2));
  sys->o_Y = ar.take((size_t)3 * sys->n_loc * sys->chunk * sizeof(double2));
  sys->o_heff = ar.take((size_t)std::max<long long>(1, sys->blk_elems) * sizeof(double2));
  sys->o_tvps = ar.take((size_t)4 * sys->nb_max * std::max(n, sys->n_states) * sizeof(double2));
  sys->o_theta_sc = ar.take((size_t)2 * sys->nb_max * std::max(sys->n_states, 1) * sizeof(double2));
  sys->o_proj = ar.take((size_t)4 * n2 * sizeof(double2));
  sys->o_tmp3 = ar.take((size_t)3 * n2 * sizeof(double2));
  sys->o_eigA = ar.take((size_t)n2 * sizeof(double2));
  sys->o_eigV = ar.take((size_t)n2 * sizeof(double2));
  sys->o_eigw = ar.take((size_t)n * sizeof(double));
  sys->o_eigwork = ar.take(jacobi_work_bytes(n));
  sys->o_k6 = ar.take((size_t)sys->nb_max * n * sizeof(double2));
  sys->o_stepslab = mm ? 0 : ar.take((size_t)std::min(sys->n_k, FFT_MAXK) * fft_rb_slab_values(sys->rgrid) * n * rb_elem(sys));
  if (mm) {
    sys->o_box_t = ar.take(mm_box_values(g) * sizeof(double2));
    sys->o_box_v = ar.take(mm_box_values(g) * sizeof(double2));
    sys->o_box_step = ar.take(mm_box_values(g) * sizeof(double2));
    sys->o_box_scr = ar.take(mm_box_scratch(g) * sizeof(double2));
  }
  sys->o_zero32 = resid32(sys) ? ar.take((size_t)sys->ngrid * sizeof(float)) : 0;
  if (sys->rb_synth) {
    const Grid &r = sys->rgrid;
    sys->o_rtw1 = ar.take(r.n1 * sizeof(double2));
    sys->o_rtw2 = ar.take(r.n2 * sizeof(double2));
    sys->o_rtw3 = ar.take(r.n3 * sizeof(double2));
    sys->o_M1 = ar.take((size_t)fft_rb_table_len(g.n1, r.n1) * sizeof(double));
    sys->o_M2 = ar.take((size_t)fft_rb_table_len(g.n2, r.n2) * sizeof(double));
    sys->o_M3 = ar.take((size_t)fft_rb_table_len(g.n3, r.n3) * sizeof(double));
    sys->o_F1 = ar.take((size_t)fft_rb_frag_len(g.n1, r.n1) * sizeof(double));
    sys->o_F2 = ar.take((size_t)fft_rb_frag_len(g.n2, r.n2) * sizeof(double));
    sys->o_F3 = ar.take((size_t)fft_rb_frag_len(g.n3, r.n3) * sizeof(double));
    sys->o_syn1 = ar.take((size_t)g.n3 * g.n2 * r.n1 * sizeof(double));
    sys->o_syn2 = ar.take((size_t)g.n3 * r.n2 * r.n1 * sizeof(double));
  }
  sys->o_subdev = ar.take(sys->n_k * sizeof(SubDev));
  {
    const int fc = std::min(1024, std::max(sys->max_cols, sys->n_states));
    sys->o_full = ar.take((size_t)8 * sys->nb_max * fc * sizeof(double2));
    sys->o_fscal = ar.take((size_t)4 * fc * sizeof(double2));
  }
  sys->o_hstep = ar.take((size_t)std::max<long long>(1, sys->blk_elems) * sizeof(double2));
  const size_t k2cap_apply = (size_t)4 * sys->n_atoms * 3 * sizeof(ZProb) + 1024;
  sys->o_k2_hs1 = ar.take(k2cap_apply);
  sys->o_k2_hs2 = ar.take(k2cap_apply);
  sys->o_k2_tv1 = ar.take(k2cap_apply);
  sys->o_k2_tv2 = ar.take(k2cap_apply);
  const size_t k2cap_step = (size_t)4 * sys->n_atoms * sys->n_k * sizeof(ZProb) + 1024;
  sys->o_k2_st1 = ar.take(k2cap_step);
  sys->o_k2_st2 = ar.take(k2cap_step);
  sys->o_vstep_tab = ar.take((size_t)sys->n_k * ((n + PROJ_BLK - 1) / PROJ_BLK) * sizeof(ZProb) + 256);
  if (resid32(sys)) {
    sys->o_k7_32 = ar.take(k2cap_step);
    sys->o_vstep32 = ar.take((size_t)sys->n_k * ((n + PROJ_BLK - 1) / PROJ_BLK) * sizeof(ZProb) + 256);
    sys->o_hstep32 = ar.take((size_t)std::max<long long>(1, sys->blk_elems) * sizeof(float2));
    sys->o_mtperm = ar.take((size_t)std::max(1, sys->n_loc) * sizeof(int));
    int r = 0;
    for (int a = 0; a < sys->n_atoms; ++a) {
      sys->mt_row32.push_back(r);
      r += sys->n_mt[a] + sys->n_lo[a];
    }
  }
  for (int k = 0; k < sys->n_k; ++k) {
    KHost &kh = sys->kh[k];
    kh.o_gk = ar.take((size_t)3 * kh.n_g * sizeof(double));
    kh.o_pptr = ar.take((size_t)(g.nbz + 1) * sizeof(int));
    kh.o_pxr = ar.take((size_t)2 * g.nbz * sizeof(int));
    kh.o_ptsg = ar.take((size_t)kh.n_g * sizeof(int));
    kh.o_ptsxy = ar.take((size_t)kh.n_g * sizeof(int));
    if (sys->ap_red) kh.o_ptsxy_a = ar.take((size_t)kh.n_g * sizeof(int));
    kh.o_subs = ar.take((size_t)4 * n2 * sizeof(double2));
    kh.o_tilde = ar.take((size_t)4 * n2 * sizeof(double2));
    kh.o_L = ar.take((size_t)n2 * sizeof(double2));
    kh.o_Linv = ar.take((size_t)n2 * sizeof(double2));
    kh.o_LH = ar.take((size_t)n2 * sizeof(double2));
    kh.o_LinvH = ar.take((size_t)n2 * sizeof(double2));
    kh.o_vstep = ar.take((size_t)n2 * sizeof(double2));
    kh.o_hm = ar.take((size_t)n2 * sizeof(double2));
    kh.o_dev = ar.take((size_t)assemble_blocks(n) * sizeof(double));
    kh.o_work = sys->h_in_lds ? 0 : ar.take((size_t)sys->n_states * n2 * sizeof(double2));
    kh.o_phit = ar.take((size_t)kh.k_ext * n * sizeof(double2));
    kh.o_yext = ar.take((size_t)kh.k_ext * n * sizeof(double2));
    kh.o_cache = mm ? 0 : ar.take(fft_rb_slab_values(sys->rgrid) * n * rb_elem(sys));
    if (mm) {
      const size_t m2 = (size_t)kh.n_g * kh.n_g * sizeof(double2);
      kh.o_gint = ar.take((size_t)3 * kh.n_g * sizeof(int));
      kh.o_mmT = ar.take(m2);
      kh.o_mmV = ar.take(m2);
      kh.o_mmP = ar.take(m2);
      kh.o_mmS = ar.take(m2);
      kh.o_mmVt = ar.take(m2);
    }
    if (resid32(sys)) {
      kh.o_phit32 = ar.take((size_t)kh.k_ext * n * sizeof(float2));
      kh.o_yext32 = ar.take((size_t)kh.k_ext * n * sizeof(float2));
    }
  }
  sys->ws_need = ar.off;
  sys->sd.assign(sys->n_k, SubDev{});
  *ws_bytes = sys->ws_need;
  *out = sys;
  return LTD_OK;
}

ltd_status ltd_bind_workspace(ltd_system *sys, void *ws, size_t bytes, void *stream) {
  if (!sys || !ws) return LTD_EINVAL;
  if (bytes < sys->ws_need) return LTD_EWORKSPACE;
  if (((uintptr_t)ws % ALIGN) != 0) return LTD_EALIGN;
  sys->ws = reinterpret_cast<char *>(ws);
  sys->ws_bound = bytes;
  hipStream_t s = S(stream);
  fft_init_attrs();
  subspace_init_attrs();
  if (!static_scratch()) return LTD_EHIP;  // the allocation-free apply's array on this device
  if (!sys->side) {
    LTD_HIP(hipStreamCreateWithFlags(&sys->side, hipStreamNonBlocking));
    LTD_HIP(hipEventCreateWithFlags(&sys->ev_fork, hipEventDisableTiming));
    LTD_HIP(hipEventCreateWithFlags(&sys->ev_join, hipEventDisableTiming));
    LTD_HIP(hipStreamCreateWithFlags(&sys->side2, hipStreamNonBlocking));
    LTD_HIP(hipEventCreateWithFlags(&sys->ev_p0, hipEventDisableTiming));
    LTD_HIP(hipEventCreateWithFlags(&sys->ev_asm, hipEventDisableTiming));
    LTD_HIP(hipEventCreateWithFlags(&sys->ev_pj, hipEventDisableTiming));
    LTD_HIP(hipStreamCreateWithFlags(&sys->side3, hipStreamNonBlocking));
    LTD_HIP(hipEventCreateWithFlags(&sys->ev_xz, hipEventDisableTiming));
    LTD_HIP(hipEventCreateWithFlags(&sys->ev_syn, hipEventDisableTiming));
  }
  // twiddles exp(-2 pi i m / L)
  auto tw = [&](int L, size_t off) -> ltd_status {
    std::vector<double2> t(L);
    for (int m = 0; m < L; ++m) {
      const double ang = -2.0 * M_PI * (double)m / (double)L;
      t[m] = make_double2(std::cos(ang), std::sin(ang));
    }
    LTD_HIP(hipMemcpy(sys->ws + off, t.data(), L * sizeof(double2), hipMemcpyHostToDevice));
    return LTD_OK;
  };
  LTD_TRY(tw(sys->n1, sys->o_tw1));
  LTD_TRY(tw(sys->n2, sys->o_tw2));
  LTD_TRY(tw(sys->n3, sys->o_tw3));
  if (sys->rb_synth) {
    const Grid &r = sys->rgrid;
    LTD_TRY(tw(r.n1, sys->o_rtw1));
    LTD_TRY(tw(r.n2, sys->o_rtw2));
    LTD_TRY(tw(r.n3, sys->o_rtw3));
    // tab[m] = (1/N) sum_{|q| <= 2b} exp(2 pi i q m / L): the axis matrix
    // M[j'][j] = (1/N) sum_{|q| <= 2b} exp(2 pi i q j'/N') exp(-2 pi i q j/N) (real)
    // at j'/N' - j/N = m/L, L = lcm(N, N')
    auto mat = [&](int np, int nn, int b, size_t off, size_t off_f) -> ltd_status {
      const int L = fft_rb_table_len(nn, np);
      std::vector<double> m(L);
      for (int e = 0; e < L; ++e) {
        double acc = 1.0;
        for (int q = 1; q <= 2 * b; ++q) acc += 2.0 * std::cos(2.0 * M_PI * (double)((long long)q * e % L) / L);
        m[e] = acc / nn;
      }
      LTD_HIP(hipMemcpy(sys->ws + off, m.data(), m.size() * sizeof(double), hipMemcpyHostToDevice));
      std::vector<double> f(fft_rb_frag_len(nn, np));
      fft_rb_frag(nn, np, m.data(), f.data());
      LTD_HIP(hipMemcpy(sys->ws + off_f, f.data(), f.size() * sizeof(double), hipMemcpyHostToDevice));
      return LTD_OK;
    };
    LTD_TRY(mat(r.n1, sys->n1, r.bx, sys->o_M1, sys->o_F1));
    LTD_TRY(mat(r.n2, sys->n2, r.by, sys->o_M2, sys->o_F2));
    LTD_TRY(mat(r.n3, sys->n3, r.bz, sys->o_M3, sys->o_F3));
  }
  for (int k = 0; k < sys->n_k; ++k) {
    KHost &kh = sys->kh[k];
    LTD_HIP(hipMemcpy(sys->ws + kh.o_gk, &sys->gk[3 * kh.g_off], 3 * kh.n_g * sizeof(double), hipMemcpyHostToDevice));
    LTD_HIP(hipMemcpy(sys->ws + kh.o_pptr, kh.plane_ptr.data(), kh.plane_ptr.size() * sizeof(int), hipMemcpyHostToDevice));
    LTD_HIP(hipMemcpy(sys->ws + kh.o_pxr, kh.plane_x.data(), kh.plane_x.size() * sizeof(int), hipMemcpyHostToDevice));
    LTD_HIP(hipMemcpy(sys->ws + kh.o_ptsg, kh.pts_g.data(), kh.n_g * sizeof(int), hipMemcpyHostToDevice));
    LTD_HIP(hipMemcpy(sys->ws + kh.o_ptsxy, kh.pts_xy.data(), kh.n_g * sizeof(int), hipMemcpyHostToDevice));
    if (sys->ap_red)
      LTD_HIP(hipMemcpy(sys->ws + kh.o_ptsxy_a, kh.pts_xy_a.data(), kh.n_g * sizeof(int), hipMemcpyHostToDevice));
    kh.bound = false;
  }
  std::vector<int> zero(16, 0);
  LTD_HIP(hipMemcpy(sys->ws + sys->o_status, zero.data(), 16 * sizeof(int), hipMemcpyHostToDevice));
  if (resid32(sys) && sys->n_loc > 0) {
    std::vector<int> perm;
    for (int a = 0; a < sys->n_atoms; ++a) {
      for (int i = 0; i < sys->n_mt[a]; ++i) perm.push_back(sys->a_off[a] + i);
      for (int q = 0; q < sys->n_lo[a]; ++q) perm.push_back(sys->n_a + sys->l_off[a] + q);
    }
    LTD_HIP(hipMemcpy(sys->ws + sys->o_mtperm, perm.data(), perm.size() * sizeof(int), hipMemcpyHostToDevice));
  }
  LTD_HIP(launch_thv(sys->at<double>(sys->o_thv), sys->theta, sys->v_r, sys->ngrid, s));
  if (sys->route == LTD_ROUTE_FFT) {
    LTD_TRY(rebuild_potential(sys, sys->v_r, nullptr, 0, sys->at<double>(sys->o_thv_rb), false, s));
    if (sys->ap_red || sys->ap_box) {
      const std::vector<double> ones(sys->ngrid, 1.0);
      LTD_HIP(hipMemcpy(sys->ws + sys->o_ones, ones.data(), ones.size() * sizeof(double), hipMemcpyHostToDevice));
    }
    if (sys->ap_red) {  // Theta and Theta V of the bound potential on the apply grid, grid order
      const auto syn = [&](const double *v, size_t off, bool plain) -> ltd_status {
        LTD_HIP(fft_rb_synth(rgrid_of(sys), sys->n1, sys->n2, sys->n3, sys->theta, v, nullptr, 0,
                             sys->at<double>(sys->o_M1), sys->at<double>(sys->o_M2), sys->at<double>(sys->o_M3),
                             sys->at<double>(sys->o_F1), sys->at<double>(sys->o_F2), sys->at<double>(sys->o_F3),
                             sys->at<double>(sys->o_syn1), sys->at<double>(sys->o_syn2), sys->at<double>(off),
                             nullptr, false, s, plain));
        return LTD_OK;
      };
      LTD_TRY(syn(sys->at<double>(sys->o_ones), sys->o_th_ap, true));
      LTD_TRY(syn(sys->v_r, sys->o_thv_ap, true));
      if (sys->ap_box) {  // the same two in the x/z kernel's layout
        LTD_TRY(syn(sys->at<double>(sys->o_ones), sys->o_th_x, false));
        LTD_TRY(syn(sys->v_r, sys->o_thv_x, false));
      }
    } else if (sys->ap_box) {  // Theta alone in the x/z layout on the grid itself
      LTD_HIP(fft_rb_thv(grid_of(sys), sys->theta, sys->at<double>(sys->o_ones), nullptr, 0,
                         sys->at<double>(sys->o_th_x), nullptr, false, s));
    }
  } else {  // the dense interstitial blocks of every k-point (natural G order)
    const Grid g = grid_of(sys);
    double2 *bt = sys->at<double2>(sys->o_box_t), *bv = sys->at<double2>(sys->o_box_v);
    LTD_HIP(mm_box_coefficients(g, sys->theta, nullptr, nullptr, 0, sys->at<double2>(sys->o_box_scr), bt, s));
    LTD_HIP(mm_box_coefficients(g, sys->theta, sys->v_r, nullptr, 0, sys->at<double2>(sys->o_box_scr), bv, s));
    for (int k = 0; k < sys->n_k; ++k) {
      KHost &kh = sys->kh[k];
      LTD_HIP(hipMemcpy(sys->ws + kh.o_gint, &sys->g_int[3 * kh.g_off], 3 * kh.n_g * sizeof(int),
                        hipMemcpyHostToDevice));
      const int *gi = sys->at<int>(kh.o_gint);
      const double *gkd = sys->at<double>(kh.o_gk);
      const size_t outs[4] = {kh.o_mmS, kh.o_mmT, kh.o_mmV, kh.o_mmP};
      for (int w = 0; w < 4; ++w)
        LTD_HIP(mm_dense(w, g, gi, gkd, nullptr, kh.n_g, bt, bv, sys->at<double2>(outs[w]), kh.n_g, s));
    }
  }
  if (resid32(sys)) LTD_HIP(hipMemsetAsync(sys->ws + sys->o_zero32, 0, sys->ngrid * sizeof(float), s));
  // K2 tables of the apply chunk
  double2 *W = sys->at<double2>(sys->o_W), *Y = sys->at<double2>(sys->o_Y);
  const long long yst = (long long)sys->n_loc * sys->chunk;
  {
    std::vector<ZProb> p1, p2;
    build_k2(sys, {sys->at<double2>(sys->o_heff), sys->o}, W, sys->n_loc, {Y, Y + yst}, sys->n_loc, sys->chunk, p1, p2);
    LTD_TRY(upload_k2(sys, p1, p2, sys->k2_hs, sys->o_k2_hs1, sys->o_k2_hs2, (size_t)4 * sys->n_atoms * 3 * sizeof(ZProb) + 1024));
  }
  {
    std::vector<ZProb> p1, p2;
    build_k2(sys, {sys->h, sys->pz, sys->o}, W, sys->n_loc, {Y, Y + yst, Y + 2 * yst}, sys->n_loc, sys->chunk, p1, p2);
    LTD_TRY(upload_k2(sys, p1, p2, sys->k2_tvps, sys->o_k2_tv1, sys->o_k2_tv2, (size_t)4 * sys->n_atoms * 3 * sizeof(ZProb) + 1024));
  }
  for (int k = 0; k < sys->n_k; ++k) {
    SubDev &d = sys->sd[k];
    d = SubDev{};
    d.kw = sys->kw[k];
  }
  sys->cheb_dt = NAN;
  sys->gvalid = false;
  LTD_HIP(hipStreamSynchronize(s));
  return LTD_OK;
}

ltd_status ltd_destroy(ltd_system *sys) {
  if (!sys) return LTD_EINVAL;
  drop_graphs(sys);
  if (sys->cap_stream) (void)hipStreamDestroy(sys->cap_stream);
  if (sys->side) (void)hipStreamDestroy(sys->side);
  if (sys->ev_fork) (void)hipEventDestroy(sys->ev_fork);
  if (sys->ev_join) (void)hipEventDestroy(sys->ev_join);
  if (sys->side2) (void)hipStreamDestroy(sys->side2);
  if (sys->ev_p0) (void)hipEventDestroy(sys->ev_p0);
  if (sys->ev_asm) (void)hipEventDestroy(sys->ev_asm);
  if (sys->ev_pj) (void)hipEventDestroy(sys->ev_pj);
  if (sys->side3) (void)hipStreamDestroy(sys->side3);
  if (sys->ev_xz) (void)hipEventDestroy(sys->ev_xz);
  if (sys->ev_syn) (void)hipEventDestroy(sys->ev_syn);
  delete sys;
  return LTD_OK;
}

ltd_status ltd_sync_status(ltd_system *sys, void *stream) {
  if (!sys) return LTD_EINVAL;
  if (!sys->ws) return LTD_ESTATE;
  int st = 0;
  LTD_TRY(read_status(sys, S(stream), &st));
  int zero[2] = {0, 0};
  LTD_HIP(hipMemcpy(sys->ws + sys->o_status, zero, sizeof(zero), hipMemcpyHostToDevice));
  return st;
}

ltd_status ltd_apply_HS(ltd_system *sys, int k, const double a_vec[3], const void *C, int ldc, int n, void *HC,
                        int ldhc, void *SC, int ldsc, void *stream) {
  if (!sys || !a_vec) return LTD_EINVAL;
  if (!sys->ws) return LTD_ESTATE;
  if (k < 0 || k >= sys->n_k || n < 0 || n > sys->max_cols) return LTD_ESHAPE;
  if (n == 0) return LTD_OK;
  if (!C || !HC || !SC) return LTD_EINVAL;
  if (!std::isfinite(a_vec[0]) || !std::isfinite(a_vec[1]) || !std::isfinite(a_vec[2])) return LTD_EINVAL;
  // only the z momentum block is part of the system: a transverse A cannot be applied
  if (a_vec[0] != 0.0 || a_vec[1] != 0.0) return LTD_EUNSUPPORTED;
  const int nb = sys->kh[k].n_basis;
  if (ldc < nb || ldhc < nb || ldsc < nb) return LTD_ESHAPE;
  if (!aligned16(C) || !aligned16(HC) || !aligned16(SC)) return LTD_EALIGN;
  if (HC == C || SC == C || HC == SC) return LTD_EINVAL;
  double2 *outs[4] = {reinterpret_cast<double2 *>(HC), reinterpret_cast<double2 *>(SC), nullptr, nullptr};
  const int ldo[4] = {ldhc, ldsc, 0, 0};
  return apply_cols(sys, k, FFT_MODE_HS, a_vec[2], reinterpret_cast<const double2 *>(C), ldc, n, outs, ldo, S(stream));
}

ltd_status ltd_propagate_full(ltd_system *sys, int k, void *C, int ldc, int n, const ltd_full_args *fa, int n_steps,
                              void *stream) {
  if (!sys || !C || !fa || !fa->a_mid) return LTD_EINVAL;
  if (!sys->ws) return LTD_ESTATE;
  if (k < 0 || k >= sys->n_k || n < 1 || n > std::min(1024, std::max(sys->max_cols, sys->n_states)) || n_steps < 0)
    return LTD_ESHAPE;
  const int nb = sys->kh[k].n_basis;
  if (ldc < nb) return LTD_ESHAPE;
  if (!aligned16(C)) return LTD_EALIGN;
  if (fa->order < 1 || fa->order > TAYLOR_MAX || !std::isfinite(fa->dt) || fa->dt == 0.0 || !std::isfinite(fa->c0) ||
      fa->cg_max_iter < 1 || !(fa->cg_tol > 0.0))
    return LTD_EINVAL;
  for (int i = 0; i < n_steps; ++i)
    if (!std::isfinite(fa->a_mid[i])) return LTD_EINVAL;
  hipStream_t s = S(stream);
  double2 *x = reinterpret_cast<double2 *>(C);
  double2 *term = full_blk(sys, 0), *acc = full_blk(sys, 1), *ht = full_blk(sys, 2), *st = full_blk(sys, 3);
  double2 *y = full_blk(sys, 4);
  double worst = 0.0;
  int most = 0;
  const int ld = sys->nb_max;
  for (int step = 0; step < n_steps; ++step) {
    const double a = fa->a_mid[step];
    LTD_HIP(launch_copy_rows(term, ld, x, ldc, nb, n, false, s));
    LTD_HIP(launch_copy_rows(acc, ld, x, ldc, nb, n, false, s));
    for (int q = 1; q <= fa->order; ++q) {
      double2 *outs[4] = {ht, st, nullptr, nullptr};
      const int ldo[4] = {ld, ld, 0, 0};
      LTD_TRY(apply_cols(sys, k, FFT_MODE_HS, a, term, ld, n, outs, ldo, s));
      double res = 0.0;
      int it = 0;
      LTD_TRY(cg_solve(sys, k, ht, n, y, fa->cg_max_iter, fa->cg_tol, &res, &it, s));
      worst = std::max(worst, res);
      most = std::max(most, it);
      // term <- (-i dt / q) (S^{-1} H term - c0 term), acc += term
      LTD_HIP(launch_taylor_term(term, y, term, make_double2(0.0, -fa->dt / q), fa->c0, acc, nb, n, ld, s));
    }
    LTD_HIP(launch_copy_rows(x, ldc, acc, ld, nb, n, false, s));
    LTD_HIP(launch_scale_block(x, make_double2(std::cos(fa->dt * fa->c0), -std::sin(fa->dt * fa->c0)), nb, n, ldc,
                               s));
  }
  LTD_HIP(hipStreamSynchronize(s));
  if (fa->cg_resid) *fa->cg_resid = worst;
  if (fa->cg_iters) *fa->cg_iters = most;
  return LTD_OK;
}

ltd_status ltd_full_spectrum(ltd_system *sys, int k, const void *x0, int iters, int cg_max_iter, double cg_tol,
                             double *eps_max, void *stream) {
  if (!sys || !x0 || !eps_max) return LTD_EINVAL;
  if (!sys->ws) return LTD_ESTATE;
  if (k < 0 || k >= sys->n_k || iters < 1 || cg_max_iter < 1 || !(cg_tol > 0.0)) return LTD_ESHAPE;
  if (!aligned16(x0)) return LTD_EALIGN;
  hipStream_t s = S(stream);
  const int nb = sys->kh[k].n_basis, ld = sys->nb_max;
  double2 *x = full_blk(sys, 0), *hx = full_blk(sys, 1), *sx = full_blk(sys, 2), *y = full_blk(sys, 3);
  double2 *sc = sys->at<double2>(sys->o_fscal);
  LTD_HIP(launch_copy_rows(x, ld, reinterpret_cast<const double2 *>(x0), nb, nb, 1, false, s));
  double lam = 0.0;
  for (int it = 0; it < iters; ++it) {
    double2 *outs[4] = {hx, sx, nullptr, nullptr};
    const int ldo[4] = {ld, ld, 0, 0};
    LTD_TRY(apply_cols(sys, k, FFT_MODE_HS, 0.0, x, ld, 1, outs, ldo, s));
    LTD_HIP(launch_col_dots(x, hx, nb, 1, ld, sc, s));
    LTD_HIP(launch_col_dots(x, sx, nb, 1, ld, sc + 1, s));
    double2 h2[2];
    LTD_HIP(hipMemcpyAsync(h2, sc, sizeof(h2), hipMemcpyDeviceToHost, s));
    LTD_HIP(hipStreamSynchronize(s));
    lam = h2[0].x / h2[1].x;
    double res = 0.0;
    int used = 0;
    LTD_TRY(cg_solve(sys, k, hx, 1, y, cg_max_iter, cg_tol, &res, &used, s));
    // x <- y / |y|
    LTD_HIP(launch_col_dots(y, y, nb, 1, ld, sc, s));
    double2 nn;
    LTD_HIP(hipMemcpyAsync(&nn, sc, sizeof(nn), hipMemcpyDeviceToHost, s));
    LTD_HIP(hipStreamSynchronize(s));
    if (!(nn.x > 0.0) || !std::isfinite(nn.x)) return LTD_ENONFINITE;
    LTD_HIP(launch_copy_rows(x, ld, y, ld, nb, 1, false, s));
    LTD_HIP(launch_scale_block(x, make_double2(1.0 / std::sqrt(nn.x), 0.0), nb, 1, ld, s));
  }
  *eps_max = lam;
  return LTD_OK;
}

ltd_status ltd_apply_HS_static(ltd_system *sys, int k, const double a_vec[3], const void *C, int ldc, int n,
                               void *HC, int ldhc, void *SC, int ldsc, void *stream) {
  if (!sys || !a_vec) return LTD_EINVAL;
  if (!sys->ws) return LTD_ESTATE;
  if (k < 0 || k >= sys->n_k || n < 0) return LTD_ESHAPE;
  if (n == 0) return LTD_OK;
  if (!C || !HC || !SC) return LTD_EINVAL;
  if (!std::isfinite(a_vec[0]) || !std::isfinite(a_vec[1]) || !std::isfinite(a_vec[2])) return LTD_EINVAL;
  if (a_vec[0] != 0.0 || a_vec[1] != 0.0) return LTD_EUNSUPPORTED;
  const int nb = sys->kh[k].n_basis;
  if (ldc < nb || ldhc < nb || ldsc < nb) return LTD_ESHAPE;
  if (!aligned16(C) || !aligned16(HC) || !aligned16(SC)) return LTD_EALIGN;
  if (HC == C || SC == C || HC == SC) return LTD_EINVAL;
  const int cmax = static_cols(sys, n);
  if (cmax < 1) return LTD_EUNSUPPORTED;  // one column's scratch exceeds LTD_STATIC_SCRATCH_BYTES
  char *base = static_scratch();
  if (!base) return LTD_EHIP;
  hipStream_t s = S(stream);
  const double2 *c = reinterpret_cast<const double2 *>(C);
  double2 *hc = reinterpret_cast<double2 *>(HC), *sc = reinterpret_cast<double2 *>(SC);
  const int ldo[4] = {ldhc, ldsc, 0, 0};
  for (int j0 = 0; j0 < n; j0 += cmax) {
    const int cols = std::min(cmax, n - j0);
    double2 *o[4] = {hc + (long long)j0 * ldhc, sc + (long long)j0 * ldsc, nullptr, nullptr};
    LTD_TRY(apply_chunk(sys, k, FFT_MODE_HS, a_vec[2], c + (long long)j0 * ldc, ldc, cols, o, ldo, s, nullptr,
                        static_bufs(sys, base, cols)));
  }
  return LTD_OK;
}

ltd_status ltd_project_subspace(ltd_system *sys, int k, const void *phi, int ldphi, int n_aux, void *h0_sub,
                                void *s_sub, const void *C, int ldc, int n_states, void *theta, void *stream) {
  if (!sys || !phi) return LTD_EINVAL;
  if (!sys->ws) return LTD_ESTATE;
  if (k < 0 || k >= sys->n_k || n_aux != sys->n_aux) return LTD_ESHAPE;
  KHost &kh = sys->kh[k];
  if (ldphi < kh.n_basis) return LTD_ESHAPE;
  if (C && (ldc < kh.n_basis || n_states != sys->n_states || !theta)) return LTD_ESHAPE;
  if (!aligned16(phi) || (h0_sub && !aligned16(h0_sub)) || (s_sub && !aligned16(s_sub)) || (C && !aligned16(C)) ||
      (theta && !aligned16(theta)))
    return LTD_EALIGN;
  hipStream_t s = S(stream);
  const int n = sys->n_aux;
  const long long n2 = (long long)n * n;
  const double2 *Phi = reinterpret_cast<const double2 *>(phi);
  LTD_TRY(setup_sub(sys, k, Phi, ldphi, s));
  int fail = 0;
  LTD_HIP(hipStreamSynchronize(s));
  LTD_HIP(hipMemcpy(&fail, sys->ws + sys->o_status + sizeof(int), sizeof(int), hipMemcpyDeviceToHost));
  if (fail) return LTD_ENOTSPD;
  double2 *subs = sys->at<double2>(kh.o_subs);
  double2 *L = sys->at<double2>(kh.o_L), *Li = sys->at<double2>(kh.o_Linv);
  const double2 one = make_double2(1.0, 0.0), zero = make_double2(0.0, 0.0);
  // Phi~ = Phi L^{-H}; Phi~_ext = [Phi~_G; A Phi~_G; Phi~_LO]
  double2 *pt = sys->at<double2>(sys->o_k6);
  LTD_TRY(gemm1(sys, OP_N, OP_C, zp(kh.n_basis, n, n, Phi, ldphi, Li, n, pt, sys->nb_max), s));
  double2 *pe = sys->at<double2>(kh.o_phit);
  LTD_HIP(launch_copy_rows(pe, kh.k_ext, pt, sys->nb_max, kh.n_g, n, false, s));
  LTD_TRY(gemm1(sys, OP_N, OP_N, zp(sys->n_a, n, kh.n_g, sys->amat + kh.amat_off, sys->n_a, pt, sys->nb_max,
                                    pe + kh.n_g, kh.k_ext), s));
  if (sys->n_lo_tot > 0)
    LTD_HIP(launch_copy_rows(pe + kh.n_g + sys->n_a, kh.k_ext, pt + kh.n_g, sys->nb_max, sys->n_lo_tot, n, false, s));
  // cached plane-wave part of Phi~, transformed along y only (box in x and z)
  if (sys->route == LTD_ROUTE_FFT) {
    FftKArgs ka{};
    ka.sph[0] = sphere_of(sys, k);
    ka.in[0].c = pe;
    ka.in[0].ldc = kh.k_ext;
    ka.slab_out[0] = sys->at<double2>(kh.o_cache);
    LTD_HIP(fft_rb_cache(rgrid_of(sys), ka, 1, n, s, resid32(sys)));
  }
  // the G rows of Phi~_ext in the order the rebuild writes Y (the sphere tables'
  // plane order, so that its writes are contiguous); the projection sums over G
  LTD_HIP(launch_gather_rows(pe, kh.k_ext, pt, sys->nb_max, sys->at<int>(kh.o_ptsg), kh.n_g, n, s));
  if (resid32(sys))  // complex64 Phi~_ext of the FP32 residual projection (atom-contiguous MT rows)
    LTD_HIP(launch_rows_to_c64(sys->at<float2>(kh.o_phit32), kh.k_ext, pe, kh.k_ext, kh.n_g,
                               sys->at<int>(sys->o_mtperm), sys->n_loc, n, s));
  // outputs in the Phi basis
  if (h0_sub) LTD_HIP(launch_axpby(reinterpret_cast<double2 *>(h0_sub), subs, subs + n2, 1.0, 1.0, n2, s));
  if (s_sub)
    LTD_HIP(hipMemcpyAsync(s_sub, subs + 3 * n2, n2 * sizeof(double2), hipMemcpyDeviceToDevice, s));
  if (C) {
    // theta = S^{-1} Phi^H (S C) = L^{-H} L^{-1} Phi^H (S C)
    double2 *hsc = sys->at<double2>(sys->o_theta_sc);
    double2 *outs[4] = {hsc, hsc + (long long)sys->nb_max * n_states, nullptr, nullptr};
    const int ldo[4] = {sys->nb_max, sys->nb_max, 0, 0};
    LTD_TRY(apply_cols(sys, k, FFT_MODE_HS, 0.0, reinterpret_cast<const double2 *>(C), ldc, n_states, outs, ldo, s));
    double2 *t1 = sys->at<double2>(sys->o_tmp3);
    double2 *t2 = t1 + (long long)n * n_states;
    LTD_TRY(gemm1(sys, OP_C, OP_N, zp(n, n_states, kh.n_basis, Phi, ldphi, outs[1], sys->nb_max, t1, n), s));
    LTD_TRY(gemm1(sys, OP_N, OP_N, zp(n, n_states, n, Li, n, t1, n, t2, n), s));
    LTD_TRY(gemm1(sys, OP_C, OP_N, zp(n, n_states, n, Li, n, t2, n, reinterpret_cast<double2 *>(theta), n), s));
  }
  (void)one;
  (void)zero;
  // spectrum of H~0 -> Chebyshev interval and critical time step
  double lmin = 0, lmax = 0;
  LTD_TRY(eig_bounds(sys, k, s, &lmin, &lmax));
  kh.lam_min = lmin;
  kh.lam_max = lmax;
  kh.phi = Phi;
  kh.ldphi = ldphi;
  SubDev &d = sys->sd[k];
  const double half = 0.5 * (lmax - lmin);
  d.tt = sys->at<double2>(kh.o_tilde);
  d.vt_ref = d.tt + n2;
  d.pt = d.tt + 2 * n2;
  d.h0t = d.tt + 3 * n2;
  d.vt_step = sys->at<double2>(kh.o_vstep);
  d.L = L;
  d.Linv = Li;
  d.LH = sys->at<double2>(kh.o_LH);
  d.LinvH = sys->at<double2>(kh.o_LinvH);
  LTD_HIP(launch_conj_transpose(L, sys->at<double2>(kh.o_LH), n, s));
  LTD_HIP(launch_conj_transpose(Li, sys->at<double2>(kh.o_LinvH), n, s));
  d.work = sys->h_in_lds ? nullptr : sys->at<double2>(kh.o_work);
  d.hm = sys->at<double2>(kh.o_hm);
  d.dev = sys->at<double>(kh.o_dev);
  d.kw = sys->kw[k];
  d.c0 = 0.5 * (lmax + lmin);
  d.margin = 0.25 * half + 0.2;
  d.r = half + d.margin;
  kh.bound = true;
  sys->cheb_dt = NAN;
  sys->gvalid = false;
  LTD_TRY(build_step_tables(sys));
  LTD_TRY(upload_subdev(sys));
  LTD_HIP(hipStreamSynchronize(s));
  return LTD_OK;
}

ltd_status ltd_ritz_basis(ltd_system *sys, int k, void *x, int ldx, double *eps, void *stream) {
  if (!sys || !x) return LTD_EINVAL;
  if (!sys->ws) return LTD_ESTATE;
  if (k < 0 || k >= sys->n_k) return LTD_ESHAPE;
  KHost &kh = sys->kh[k];
  if (ldx < kh.n_basis) return LTD_ESHAPE;
  if (!aligned16(x)) return LTD_EALIGN;
  hipStream_t s = S(stream);
  const int n = sys->n_aux;
  const long long n2 = (long long)n * n;
  double2 *X = reinterpret_cast<double2 *>(x);
  const bool was_bound = kh.bound;
  LTD_TRY(setup_sub(sys, k, X, ldx, s));
  int fail = 0;
  LTD_HIP(hipStreamSynchronize(s));
  LTD_HIP(hipMemcpy(&fail, sys->ws + sys->o_status + sizeof(int), sizeof(int), hipMemcpyDeviceToHost));
  if (fail) return LTD_ENOTSPD;
  double2 *A = sys->at<double2>(sys->o_eigA), *V = sys->at<double2>(sys->o_eigV);
  double *w = sys->at<double>(sys->o_eigw);
  LTD_HIP(hipMemcpyAsync(A, sys->at<double2>(kh.o_tilde) + 3 * n2, n2 * sizeof(double2), hipMemcpyDeviceToDevice, s));
  LTD_HIP(launch_jacobi(A, V, w, n, s, sys->ws + sys->o_eigwork));
  // X <- X L^{-H} W
  double2 *t = sys->at<double2>(sys->o_k6);
  LTD_TRY(gemm1(sys, OP_N, OP_C, zp(kh.n_basis, n, n, X, ldx, sys->at<double2>(kh.o_Linv), n, t, sys->nb_max), s));
  LTD_TRY(gemm1(sys, OP_N, OP_N, zp(kh.n_basis, n, n, t, sys->nb_max, V, n, X, ldx), s));
  if (eps) LTD_HIP(hipMemcpyAsync(eps, w, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  LTD_HIP(hipStreamSynchronize(s));
  // the k-point's slots were overwritten: the previous binding (if any) is gone
  if (was_bound) kh.bound = false;
  sys->gvalid = false;
  return LTD_OK;
}

ltd_status ltd_autotune(ltd_system *sys, int *choice, double *times_us, void *stream) {
  if (!sys || !choice) return LTD_EINVAL;
  if (!sys->ws) return LTD_ESTATE;
  for (int k = 0; k < sys->n_k; ++k)
    if (!sys->kh[k].bound) return LTD_ESTATE;
  hipStream_t s = S(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  LTD_HIP(hipEventCreate(&e0));
  LTD_HIP(hipEventCreate(&e1));
  constexpr int REPS = 5;
  const auto timed = [&](auto &&launch, double *us) -> ltd_status {
    LTD_TRY(launch());  // warm-up
    LTD_HIP(hipEventRecord(e0, s));
    for (int r = 0; r < REPS; ++r) LTD_TRY(launch());
    LTD_HIP(hipEventRecord(e1, s));
    LTD_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    LTD_HIP(hipEventElapsedTime(&ms, e0, e1));
    *us = 1e3 * ms / REPS;
    return LTD_OK;
  };
  ltd_status st = LTD_OK;
  int ti = 0;
  // 1. launch shape of the x/z rebuild kernel, on the cached grid images of the
  //    first k-points and the reference potential
  const Grid g = rgrid_of(sys);
  const bool r32 = resid32(sys);
  const int n = sys->n_aux, nk = std::min(FFT_MAXK, sys->n_k);
  FftKArgs ka{};
  for (int i = 0; i < nk; ++i) {
    ka.sph[i] = sphere_of(sys, i);
    ka.slab_in[i] = sys->at<double2>(sys->kh[i].o_cache);
    ka.slab_out[i] = reinterpret_cast<double2 *>(sys->ws + sys->o_stepslab +
                                                 (size_t)i * fft_rb_slab_values(g) * n * rb_elem(sys));
  }
  const void *thv = r32 ? static_cast<const void *>(sys->at<float>(sys->o_zero32))
                        : static_cast<const void *>(sys->at<double>(sys->o_thv_rb));
  int best_v = 0;
  double best_t = 1e300;
  const int n_shapes = sys->route == LTD_ROUTE_FFT ? fft_rb_variants(g, r32) : 0;
  for (int v = 0; v < n_shapes && st == LTD_OK; ++v) {
    double us = 0.0;
    st = timed([&]() -> ltd_status {
      LTD_HIP(fft_rb_step(g, ka, nk, n, thv, s, 0, r32, v));
      return LTD_OK;
    }, &us);
    if (times_us) times_us[ti++] = us;
    if (us < best_t) best_t = us, best_v = v;
  }
  // 2. block target of the projection GEMM's K split
  const int targets[4] = {256, 512, 1024, 2048};
  int best_g = sys->vproj_target;
  best_t = 1e300;
  for (int q = 0; q < 4 && st == LTD_OK; ++q) {
    sys->vproj_target = targets[q];
    st = build_step_tables(sys);
    if (st != LTD_OK) break;
    double us = 0.0;
    st = timed([&]() -> ltd_status {
      LTD_TRY(project_v(sys, s));
      return LTD_OK;
    }, &us);
    if (times_us) times_us[ti++] = us;
    if (us < best_t) best_t = us, best_g = targets[q];
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  LTD_TRY(st);
  sys->vproj_target = best_g;
  LTD_TRY(build_step_tables(sys));
  sys->rb_variant = best_v;
  sys->gvalid = false;  // a captured step graph holds the previous shapes
  choice[0] = best_v;
  choice[1] = best_g;
  choice[2] = n_shapes;
  return LTD_OK;
}

ltd_status ltd_set_tuning(ltd_system *sys, const int *choice) {
  if (!sys || !choice) return LTD_EINVAL;
  if (choice[0] < 0 || choice[0] >= fft_rb_variants(rgrid_of(sys), resid32(sys))) return LTD_EINVAL;
  if (choice[1] < 64 || choice[1] > 8192) return LTD_EINVAL;
  sys->rb_variant = choice[0];
  if (choice[1] != sys->vproj_target) {
    sys->vproj_target = choice[1];
    if (sys->ws) LTD_TRY(build_step_tables(sys));
  }
  sys->gvalid = false;
  return LTD_OK;
}

ltd_status ltd_state_drift(ltd_system *sys, void *theta, int reorthonormalize, double *drift, void *stream) {
  if (!sys || !theta || !drift) return LTD_EINVAL;
  if (!sys->ws) return LTD_ESTATE;
  for (int k = 0; k < sys->n_k; ++k)
    if (!sys->kh[k].bound) return LTD_ESTATE;
  if (!aligned16(theta)) return LTD_EALIGN;
  hipStream_t s = S(stream);
  const int n = sys->n_aux, ns = sys->n_states;
  const long long n2 = (long long)n * n;
  double2 *X = sys->at<double2>(sys->o_tmp3);  // n x ns: S theta, then theta G^{-1/2}
  double2 *G = X + n2;                          // ns x ns: theta^H S theta
  double2 *B = G + n2;                          // ns x ns: V diag(w^{-1/2}), then G^{-1/2}
  double2 *A = sys->at<double2>(sys->o_eigA), *V = sys->at<double2>(sys->o_eigV);
  double *w = sys->at<double>(sys->o_eigw);
  std::vector<double2> gh((size_t)ns * ns);
  double worst = 0.0;
  for (int k = 0; k < sys->n_k; ++k) {
    const KHost &kh = sys->kh[k];
    double2 *th = reinterpret_cast<double2 *>(theta) + (long long)k * n * ns;
    const double2 *ssub = sys->at<double2>(kh.o_subs) + 3 * n2;
    LTD_TRY(gemm1(sys, OP_N, OP_N, zp(n, ns, n, ssub, n, th, n, X, n), s));
    LTD_TRY(gemm1(sys, OP_C, OP_N, zp(ns, ns, n, th, n, X, n, G, ns), s));
    LTD_HIP(hipMemcpyAsync(gh.data(), G, gh.size() * sizeof(double2), hipMemcpyDeviceToHost, s));
    LTD_HIP(hipStreamSynchronize(s));
    for (int j = 0; j < ns; ++j)
      for (int i = 0; i < ns; ++i) {
        const double2 g = gh[(size_t)i + (size_t)j * ns];
        worst = std::max(worst, std::hypot(g.x - (i == j ? 1.0 : 0.0), g.y));
      }
    if (reorthonormalize) {  // Loewdin: theta <- theta G^{-1/2}, G = V diag(w) V^H
      LTD_HIP(hipMemcpyAsync(A, G, (size_t)ns * ns * sizeof(double2), hipMemcpyDeviceToDevice, s));
      LTD_HIP(launch_jacobi(A, V, w, ns, s, sys->ws + sys->o_eigwork));
      LTD_HIP(launch_scale_cols(B, V, w, ns, s));
      LTD_TRY(gemm1(sys, OP_N, OP_C, zp(ns, ns, ns, B, ns, V, ns, G, ns), s));
      LTD_TRY(gemm1(sys, OP_N, OP_N, zp(n, ns, ns, th, n, G, ns, X, n), s));
      LTD_HIP(hipMemcpyAsync(th, X, (size_t)n * ns * sizeof(double2), hipMemcpyDeviceToDevice, s));
    }
  }
  LTD_HIP(hipStreamSynchronize(s));
  *drift = worst;
  return LTD_OK;
}

ltd_status ltd_rebuild_grid(const ltd_system *sys, int *lengths) {
  if (!sys || !lengths) return LTD_EINVAL;
  lengths[0] = sys->rgrid.n1;
  lengths[1] = sys->rgrid.n2;
  lengths[2] = sys->rgrid.n3;
  return LTD_OK;
}

ltd_status ltd_subspace_info(ltd_system *sys, int k, double *eps_min, double *eps_max, double *dt_cr) {
  if (!sys) return LTD_EINVAL;
  if (k < 0 || k >= sys->n_k) return LTD_ESHAPE;
  const KHost &kh = sys->kh[k];
  if (!kh.bound) return LTD_ESTATE;
  if (eps_min) *eps_min = kh.lam_min;
  if (eps_max) *eps_max = kh.lam_max;
  if (dt_cr) *dt_cr = 0.2 / (kh.lam_max - kh.lam_min);
  return LTD_OK;
}

ltd_status ltd_propagate_step(ltd_system *sys, const ltd_step_args *a, void *stream) {
  LTD_TRY(check_step_args(sys, a));
  LTD_TRY(prepare_dt(sys, a->dt));
  return step_once(sys, a, S(stream));
}

ltd_status ltd_propagate(ltd_system *sys, const ltd_step_args *a, int n_steps, void *stream) {
  LTD_TRY(check_step_args(sys, a));
  if (n_steps < 0) return LTD_ESHAPE;
  if (n_steps == 0) return LTD_OK;
  LTD_TRY(prepare_dt(sys, a->dt));
  hipStream_t s = S(stream);
  LTD_TRY(refresh_step_tables(sys, a));
  const bool pipe = a->mode == LTD_STEP_REBUILD && sys->side2 != nullptr && sys->route == LTD_ROUTE_FFT;
  if (pipe) {  // V~ of the first step, Theta V of the second, the step-index bounds of this call
    int *rs = sys->at<int>(sys->o_status) + 12;
    LTD_HIP(launch_lookahead_init(a->step, n_steps, rs, s));
    ltd_step_args a0 = *a;
    a0.step = rs;
    LTD_TRY(rebuild_v(sys, &a0, s));
    if (a->v_r_t) {
      LTD_HIP(launch_lookahead(rs + 2, s));
      LTD_TRY(rebuild_potential(sys, a->v_r_t, a->v_stride ? rs + 2 : nullptr, a->v_stride,
                                sys->at<double>(sys->o_thv_step), resid32(sys), s));
    }
  }
  LTD_TRY(ensure_graphs(sys, a, n_steps, pipe));
  int left = n_steps;
  for (int t = 0; t < GRAPH_TIERS; ++t) {
    const int reps = left / GRAPH_STEPS[t];
    if (reps == 0) continue;
    for (int i = 0; i < reps; ++i) LTD_HIP(hipGraphLaunch(sys->gexec[t], s));
    left -= reps * GRAPH_STEPS[t];
  }
  if (pipe) LTD_TRY(project_v(sys, s, 2));  // V~ of the step after the call's last
  return LTD_OK;
}

ltd_status ltd_propagate_prepare(ltd_system *sys, const ltd_step_args *a, int n_steps, void *stream) {
  (void)stream;
  LTD_TRY(check_step_args(sys, a));
  if (n_steps < 0) return LTD_ESHAPE;
  if (n_steps == 0) return LTD_OK;
  LTD_TRY(prepare_dt(sys, a->dt));
  LTD_TRY(refresh_step_tables(sys, a));
  return ensure_graphs(sys, a, n_steps,
                       a->mode == LTD_STEP_REBUILD && sys->side2 != nullptr && sys->route == LTD_ROUTE_FFT);
}

ltd_status ltd_pulse_loss(ltd_system *sys, const double *dmu, int n_steps, double *loss, void *stream) {
  if (!sys || !dmu || !loss) return LTD_EINVAL;
  if (n_steps < 0) return LTD_ESHAPE;
  LTD_HIP(launch_pulse_loss(dmu, n_steps, sys->omega, loss, S(stream)));
  return LTD_OK;
}

ltd_status ltd_propagate_step_adjoint(ltd_system *sys, const ltd_adjoint_args *aa, void *stream) {
  if (!aa) return LTD_EINVAL;
  const ltd_step_args *a = aa->fwd;
  LTD_TRY(check_step_args(sys, a));
  if (a->taylor_order != 0) return LTD_EUNSUPPORTED;  // the adjoint differentiates the exponential
  if (!aa->mu_out || (!aa->terminal && (!aa->mu_next || !aa->dl_da_mid)) || !aa->dl_da_t) return LTD_EINVAL;
  if (aa->n_steps < 1 || aa->n < 0 || aa->n > aa->n_steps || (!aa->terminal && aa->n == aa->n_steps))
    return LTD_ESHAPE;
  if (!aligned16(aa->mu_out) || (aa->mu_next && !aligned16(aa->mu_next))) return LTD_EALIGN;
  LTD_TRY(prepare_dt(sys, a->dt));
  hipStream_t s = S(stream);
  if (a->mode == LTD_STEP_REBUILD && !aa->terminal) LTD_TRY(rebuild_v(sys, a, s, nullptr, aa->n));
  AdjCtx ac{};
  ac.n = aa->n;
  ac.terminal = aa->terminal;
  ac.n_steps = aa->n_steps;
  ac.mu_next = reinterpret_cast<const double2 *>(aa->mu_next);
  ac.mu_out = reinterpret_cast<double2 *>(aa->mu_out);
  ac.dl_da_mid = aa->dl_da_mid;
  ac.dl_da_t = aa->dl_da_t;
  LTD_HIP(launch_adjoint(step_ctx(sys, a), ac, s));
  return LTD_OK;
}

ltd_status ltd_profile_steps(ltd_system *sys, const ltd_step_args *a, int n_steps, double *stage_ms,
                             void *stream) {
  LTD_TRY(check_step_args(sys, a));
  if (!stage_ms) return LTD_EINVAL;
  if (n_steps < 1) return LTD_ESHAPE;
  LTD_TRY(prepare_dt(sys, a->dt));
  hipStream_t s = S(stream);
  for (int i = 0; i < LTD_PROFILE_STAGES; ++i) stage_ms[i] = 0.0;
  for (int it = 0; it < n_steps; ++it) {
    Prof pf;
    LTD_TRY(pf.begin(s));
    LTD_TRY(step_once(sys, a, s, &pf));
    LTD_TRY(pf.collect(stage_ms, LTD_PROFILE_STAGES));
  }
  for (int i = 0; i < LTD_PROFILE_STAGES; ++i) stage_ms[i] /= n_steps;
  stage_ms[1] /= PROF_XZ_REPS;
  return LTD_OK;
}

ltd_status ltd_profile_apply(ltd_system *sys, int k, const void *C, int ldc, int n, void *HC, void *SC, int ldo,
                             double *stage_ms, void *stream) {
  if (!sys || !C || !HC || !SC || !stage_ms) return LTD_EINVAL;
  if (!sys->ws) return LTD_ESTATE;
  if (k < 0 || k >= sys->n_k || n < 1 || n > sys->max_cols) return LTD_ESHAPE;
  const int nb = sys->kh[k].n_basis;
  if (ldc < nb || ldo < nb) return LTD_ESHAPE;
  if (!aligned16(C) || !aligned16(HC) || !aligned16(SC)) return LTD_EALIGN;
  hipStream_t s = S(stream);
  for (int i = 0; i < LTD_PROFILE_STAGES; ++i) stage_ms[i] = 0.0;
  double2 *outs[4] = {reinterpret_cast<double2 *>(HC), reinterpret_cast<double2 *>(SC), nullptr, nullptr};
  const int lo[4] = {ldo, ldo, 0, 0};
  const double2 *c = reinterpret_cast<const double2 *>(C);
  for (int j0 = 0; j0 < n; j0 += sys->chunk) {
    const int cols = std::min(sys->chunk, n - j0);
    double2 *o[4] = {outs[0] + (long long)j0 * ldo, outs[1] + (long long)j0 * ldo, nullptr, nullptr};
    Prof pf;
    LTD_TRY(pf.begin(s));
    LTD_TRY(apply_chunk(sys, k, FFT_MODE_HS, 0.0, c + (long long)j0 * ldc, ldc, cols, o, lo, s, &pf,
                        workspace_bufs(sys)));
    LTD_TRY(pf.collect(stage_ms, LTD_PROFILE_STAGES));
  }
  return LTD_OK;
}

ltd_status ltd_knot_samples(const double *knots, int n_knots, double t_end, double dt, int n_steps, double *a_t,
                            double *a_mid, void *stream) {
  if (!knots || !a_t || !a_mid) return LTD_EINVAL;
  if (n_knots < 2 || n_steps < 1 || !(t_end > 0.0) || !(dt > 0.0)) return LTD_ESHAPE;
  LTD_HIP(launch_knot_samples(knots, n_knots, t_end, dt, n_steps, a_t, a_mid, S(stream)));
  return LTD_OK;
}

ltd_status ltd_knot_gradient(const double *dl_da_t, const double *dl_da_mid, int n_steps, double dt, int n_knots,
                             double t_end, double *dl_dq, void *stream) {
  if (!dl_da_t || !dl_da_mid || !dl_dq) return LTD_EINVAL;
  if (n_knots < 2 || n_steps < 1 || !(t_end > 0.0) || !(dt > 0.0)) return LTD_ESHAPE;
  LTD_HIP(launch_knot_gradient(dl_da_t, dl_da_mid, n_steps, dt, n_knots, t_end, dl_dq, S(stream)));
  return LTD_OK;
}

ltd_status ltd_chebyshev_coefficients(double tau, int kmax, double *coef, int *degree) {
  if (!coef || !degree || !std::isfinite(tau)) return LTD_EINVAL;
  if (kmax < 1 || kmax > 4096) return LTD_ESHAPE;
  std::vector<double2> c;
  *degree = cheb_coef(tau, kmax, c);
  for (int k = 0; k <= kmax; ++k) {
    coef[2 * k] = c[k].x;
    coef[2 * k + 1] = c[k].y;
  }
  return LTD_OK;
}

}  // extern "C"
