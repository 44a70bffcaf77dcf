// Host side of the C ABI declared in include/afqmc.h: argument validation,
// device-resident Hamiltonian / trial set-up, walker-workspace layout and the
// per-step kernel chain of the phaseless AFQMC walker update.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <map>
#include <string>
#include <type_traits>
#include <vector>

#include "afqmc.h"
#include "kernels.hpp"

namespace {

thread_local std::string g_err;

afqmc_status fail(afqmc_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define AFQ_CK(x)                                                                           \
  do {                                                                                      \
    hipError_t e_ = (x);                                                                    \
    if (e_ != hipSuccess)                                                                   \
      return fail(AFQMC_ERR_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_));       \
  } while (0)

int round_up(int x, int m) { return ((x + m - 1) / m) * m; }

// Device allocations owned by one library object.
struct Arena {
  std::vector<void*> ptrs;
  hipError_t alloc(void** p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) bytes = 256;
    hipError_t e = hipMalloc(p, bytes);
    if (e == hipSuccess) ptrs.push_back(*p);
    return e;
  }
  void release() {
    for (void* p : ptrs) (void)hipFree(p);
    ptrs.clear();
  }
};

bool symmetric(const double* a, int M, double tol) {
  double mx = 0.0;
  for (int i = 0; i < M * M; ++i) mx = std::max(mx, std::fabs(a[i]));
  const double lim = tol * std::max(mx, 1.0);
  for (int i = 0; i < M; ++i)
    for (int j = i + 1; j < M; ++j)
      if (!(std::fabs(a[i * M + j] - a[j * M + i]) <= lim)) return false;
  return true;
}

bool all_finite(const double* a, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

// Cyclic Jacobi eigendecomposition of a symmetric n x n matrix (row-major).
void jacobi_eigh(int n, std::vector<double> A, std::vector<double>& V, std::vector<double>& d) {
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  double fro = 0.0;
  for (double x : A) fro += x * x;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += A[(size_t)p * n + q] * A[(size_t)p * n + q];
    if (off <= 1e-34 * fro || off == 0.0) break;
    for (int p = 0; p < n; ++p) {
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[(size_t)p * n + q];
        if (apq == 0.0) continue;
        const double tau = (A[(size_t)q * n + q] - A[(size_t)p * n + p]) / (2.0 * apq);
        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        for (int k = 0; k < n; ++k) {
          const double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
          A[(size_t)k * n + p] = c * akp - s * akq;
          A[(size_t)k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          const double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
          A[(size_t)p * n + k] = c * apk - s * aqk;
          A[(size_t)q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
          V[(size_t)k * n + p] = c * vkp - s * vkq;
          V[(size_t)k * n + q] = s * vkp + c * vkq;
        }
      }
    }
  }
  d.resize(n);
  for (int i = 0; i < n; ++i) d[i] = A[(size_t)i * n + i];
}

}  // namespace

struct KernelTimer {
  unsigned mask = 0;  // bit c: time class c
  std::vector<hipEvent_t> pool;
  struct Pending { int cls; hipEvent_t a, b; };
  std::vector<Pending> pending;
  double total_ms[AFQMC_NUM_KERNEL_CLASSES] = {0};
  int64_t count[AFQMC_NUM_KERNEL_CLASSES] = {0};
  // create events ahead of a timed region (none are created inside it while
  // the pool lasts)
  void reserve(size_t n) {
    while (pool.size() < n) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) return;
      pool.push_back(e);
    }
  }
  hipEvent_t take() {
    if (pool.empty()) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      return e;
    }
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipError_t drain() {
    hipError_t err = hipSuccess;
    for (auto& p : pending) {
      float ms = 0.f;
      hipError_t e = hipEventSynchronize(p.b);
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, p.a, p.b);
      if (e == hipSuccess) {
        total_ms[p.cls] += ms;
        count[p.cls] += 1;
      } else {
        err = e;
      }
      pool.push_back(p.a);
      pool.push_back(p.b);
    }
    pending.clear();
    return err;
  }
  ~KernelTimer() {
    for (auto& p : pending) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

// Brackets one kernel launch with events when timing is enabled.
struct TimedLaunch {
  KernelTimer* t;
  int cls;
  hipStream_t st;
  hipEvent_t a = nullptr, b = nullptr;
  TimedLaunch(KernelTimer* t_, int cls_, hipStream_t st_) : t(t_), cls(cls_), st(st_) {
    if (t && ((t->mask >> cls) & 1u)) {
      a = t->take();
      b = t->take();
      if (a && b) (void)hipEventRecord(a, st);
    }
  }
  ~TimedLaunch() {
    if (a && b) {
      (void)hipEventRecord(b, st);
      t->pending.push_back({cls, a, b});
    }
  }
};

enum { KC_EXCHANGE = 0, KC_ABUILD = 1, KC_TAYLOR = 2, KC_OVERLAP = 3, KC_MGS = 4, KC_COMB = 5, KC_OTHER = 6,
       KC_FBIAS = 7 };

struct afqmc_ham {
  KernelTimer timer;
  int device = 0;
  int M = 0, G = 0;
  double e_core = 0.0;
  size_t max_lds = 65536;
  double* h = nullptr;   // [M][M]
  double* L = nullptr;   // [G][M][M]
  float* Lf = nullptr;   // [G][M][M]
  // upper triangles of the symmetric L_g, [G][M (M + 1) / 2] (row i: columns
  // i .. M - 1): the propagator build of the fused propagation writes A in
  // the same packed form (half the GEMM and half its output)
  double* Lp = nullptr;
  float* Lpf = nullptr;
  void* Lbf = nullptr;   // [G][M][M] bf16
  void* Lbf_lo = nullptr;  // [G][M][M] bf16, second term of the split (BF16X3)
  double* L2 = nullptr;  // sum_g L_g L_g
  std::vector<double> h_host;
  Arena arena;
};

struct B1Entry {
  double dt;
  std::vector<double> h64;
  std::vector<float> h32;
  double* d64;
  float* d32;
};

struct afqmc_trial {
  afqmc_ham* ham = nullptr;
  int nel[2] = {0, 0};
  int NP[2] = {16, 16};
  int MP4 = 4;
  int Nt = 0;
  double* C[2] = {nullptr, nullptr};
  double* htil[2] = {nullptr, nullptr};
  double* Lt64[2] = {nullptr, nullptr};
  float* Lt32[2] = {nullptr, nullptr};
  double* Apk64[2] = {nullptr, nullptr};  // NP <= 32: exchange A operand, repacked
  float* Apk32[2] = {nullptr, nullptr};
  void* Ltbf[2] = {nullptr, nullptr};  // bf16, fragment order of pack_ltilde_bf16
  void* Ltbf_lo[2] = {nullptr, nullptr};  // the split's second terms (BF16X3)
  int MP32 = 32;
  double* lbar = nullptr;
  double* D0 = nullptr;
  // hybrid weights: E_0 = e_core - 1/2 sum lbar^2, and (single determinant)
  // the force-bias operand Lq[k][g] = Ltil_g[a][m] at the split index k of
  // (spin, m, a): spin 0's (m a) -> m N_up + a padded to Kp[0], then spin 1's
  double e0_shift = 0.0;
  int Kp[2] = {0, 0};
  int Gp = 0;
  double* Lq64 = nullptr;  // [Kp0 + Kp1][Gp], zero padded
  float* Lq32 = nullptr;
  // exchange through Q[(n a)][(m b)] = sum_g Ltil_g[a][m] Ltil_g[b][n] per spin
  // (single determinant, when the Cholesky count makes it the cheaper route)
  bool qroute = false;  // measurements take the Q route
  bool qbuilt = false;  // Q64 / qsegs are set up
  bool q32 = false;     // Q32 / Lq32 too: the FP32 contractions are allowed (q_fp32_ok)
  double* Q64[2] = {nullptr, nullptr};  // [Kp][Kp], zero padded
  float* Q32[2] = {nullptr, nullptr};
  int4* qsegs = nullptr;  // (spin, I, J0, J1) tile-pair segments, spin 0 first
  int nseg[2] = {0, 0};
  std::vector<double> H1p;
  std::vector<B1Entry> b1;
  int n_det = 1;
  std::vector<double> coeff;
  std::vector<int32_t> exc;
  // multi-determinant trial: [n_det][2][5] (E, hole0, hole1, particle0, particle1),
  // coefficients, and per spin (L_g C) for g < G plus (h C) at g = G, [G+1][M][M]
  int* d_exc = nullptr;
  double* d_coeff = nullptr;
  double* LC64[2] = {nullptr, nullptr};
  float* LC32[2] = {nullptr, nullptr};
  // compact rows of the FP32 energy kernel (md_rows: the tables exist)
  bool md_rows = false;
  int mdKS = 0, mdR[2] = {0, 0}, mdRP[2] = {0, 0}, mdnp[2] = {0, 0};
  float* LCc[2] = {nullptr, nullptr};
  int* d_mdpair[2] = {nullptr, nullptr};
  int* d_mdpbeg[2] = {nullptr, nullptr};
  int* d_mddx = nullptr;
  double ref_ls[2] = {0, 0}, ref_el[2] = {0, 0};
  double* vref_re = nullptr;
  double* vref_im = nullptr;
  Arena arena;
};

namespace {

// Walker workspace layout (all offsets 256-byte aligned).
struct WS {
  double *th_re, *th_im;
  double *ld_re, *ld_im, *e1_re, *e1_im, *exx_re, *exx_im;
  double *vs_re, *vs_im;
  double *v_re, *v_im;
  double *lsn_re, *lsn_im, *eln_re, *eln_im, *mf_re, *mf_im, *hy_re, *hy_im;
  int *vfin, *dead, *parent;
  double *cbuf, *scal;
  double *c0_re, *c0_im, *tot_re, *tot_im;
  void* coefT;
  void* A;
  double *P_re, *P_im, *ACC_re, *ACC_im;
  void *Ta_re, *Ta_im, *Tb_re, *Tb_im;
  double* snap;
  size_t total;
};

// Doubles per walker in each of ws.ACC_re / ws.ACC_im.
long acc_cap(long M, long G, long Nt) { return std::max(M * Nt, G); }

WS layout_dims(long M, long G, long Nt, int n_det, int W, void* base) {
  WS ws;
  size_t off = 0;
  char* b = (char*)base;
  auto take = [&](size_t bytes) -> void* {
    void* p = b ? (void*)(b + off) : nullptr;
    off += (bytes + 255) & ~(size_t)255;
    return p;
  };
  const size_t wm = (size_t)W * M * Nt * sizeof(double);
  ws.th_re = (double*)take(wm);
  ws.th_im = (double*)take(wm);
  ws.ld_re = (double*)take(2 * W * sizeof(double));
  ws.ld_im = (double*)take(2 * W * sizeof(double));
  ws.e1_re = (double*)take(2 * W * sizeof(double));
  ws.e1_im = (double*)take(2 * W * sizeof(double));
  ws.exx_re = (double*)take(2 * W * sizeof(double));
  ws.exx_im = (double*)take(2 * W * sizeof(double));
  ws.vs_re = (double*)take(2 * (size_t)W * G * sizeof(double));
  ws.vs_im = (double*)take(2 * (size_t)W * G * sizeof(double));
  ws.v_re = (double*)take((size_t)W * G * sizeof(double));
  ws.v_im = (double*)take((size_t)W * G * sizeof(double));
  ws.lsn_re = (double*)take(W * sizeof(double));
  ws.lsn_im = (double*)take(W * sizeof(double));
  ws.hy_re = (double*)take(W * sizeof(double));
  ws.hy_im = (double*)take(W * sizeof(double));
  ws.eln_re = (double*)take(W * sizeof(double));
  ws.eln_im = (double*)take(W * sizeof(double));
  ws.mf_re = (double*)take(W * sizeof(double));
  ws.mf_im = (double*)take(W * sizeof(double));
  ws.vfin = (int*)take(W * sizeof(int));
  ws.dead = (int*)take(W * sizeof(int));
  ws.parent = (int*)take(W * sizeof(int));
  ws.cbuf = (double*)take(W * sizeof(double));
  ws.scal = (double*)take(16 * sizeof(double));
  ws.coefT = take((size_t)((G + 63) / 64 * 64) * 2 * W * sizeof(double));
  ws.A = take((size_t)W * 2 * M * M * sizeof(double));
  // P_*: also the split Theta of the Q route (M Nt + 128 per walker);
  // ACC_*: also the force-bias and quadratic-form partials
  const size_t wq = (size_t)W * (M * Nt + 128) * sizeof(double);
  const size_t wa = (size_t)W * acc_cap(M, G, Nt) * sizeof(double);
  ws.P_re = (double*)take(wq);
  ws.P_im = (double*)take(wq);
  ws.ACC_re = (double*)take(wa);
  ws.ACC_im = (double*)take(wa);
  ws.Ta_re = take(wm);
  ws.Ta_im = take(wm);
  ws.Tb_re = take(wm);
  ws.Tb_im = take(wm);
  ws.snap = (double*)take(wm * 2 + (size_t)W * (4 + 2 * G) * sizeof(double));
  const size_t nd = n_det > 1 ? (size_t)n_det : 0;
  ws.c0_re = (double*)take((size_t)W * 2 * nd * sizeof(double));
  ws.c0_im = (double*)take((size_t)W * 2 * nd * sizeof(double));
  ws.tot_re = (double*)take(W * sizeof(double));
  ws.tot_im = (double*)take(W * sizeof(double));
  ws.total = off;
  return ws;
}

WS layout(const afqmc_trial* tr, int W, void* base) {
  return layout_dims(tr->ham->M, tr->ham->G, tr->Nt, tr->n_det, W, base);
}

afqmc_status check_walkers(const afqmc_trial* tr, const afqmc_walkers* wk) {
  if (!wk) return fail(AFQMC_ERR_ARG, "walkers is NULL");
  if (wk->n_walkers < 1) return fail(AFQMC_ERR_ARG, "n_walkers must be >= 1");
  if (wk->system_id < 0) return fail(AFQMC_ERR_ARG, "system_id must be >= 0");
  if (!wk->phi_re || !wk->phi_im || !wk->weight || !wk->logovlp_re || !wk->logovlp_im ||
      !wk->eloc_re || !wk->eloc_im || !wk->workspace)
    return fail(AFQMC_ERR_ARG, "a walker buffer is NULL");
  const WS ws = layout(tr, wk->n_walkers, nullptr);
  if (wk->workspace_bytes < ws.total)
    return fail(AFQMC_ERR_ARG, "workspace_bytes smaller than afqmc_walker_workspace_bytes");
  return AFQMC_OK;
}

// The Q route for the exchange energy: single determinant, at least twice as
// many Cholesky vectors as orbitals (it then needs G / M times fewer flops
// than the Ltil route) and Q (M N x M N per spin) of at most 16384^2 entries.
int qpad(long K) { return (int)((K + 63) / 64 * 64); }

// Segments of the upper-triangular 64 x 64 tile pairs (I <= J) of both
// spins: row I of spin s split into runs of at most S column tiles.  S is
// chosen so that the partials (2 doubles per segment and walker) fit the
// workspace; returns the segment count per spin or false.
bool q_plan(int M, int G, int n_up, int n_dn, std::vector<int4>* segs, int nseg[2]) {
  const int nel[2] = {n_up, n_dn};
  int nt[2];
  for (int s = 0; s < 2; ++s) nt[s] = qpad((long)M * nel[s]) / 64;
  const long cap = (long)M * (n_up + n_dn);  // doubles per walker in ws.Ta_re
  for (int S = std::max(4, std::min(16, (std::max(nt[0], nt[1]) + 4) / 5)); ; S *= 2) {
    long tot = 0;
    for (int s = 0; s < 2; ++s) {
      nseg[s] = 0;
      for (int I = 0; I < nt[s]; ++I) nseg[s] += (nt[s] - I + S - 1) / S;
      tot += nseg[s];
    }
    if (2 * tot <= cap) {
      if (segs) {
        segs->clear();
        for (int s = 0; s < 2; ++s)
          for (int I = 0; I < nt[s]; ++I)
            for (int J = I; J < nt[s]; J += S) segs->push_back(make_int4(s, I, J, std::min(J + S, nt[s])));
      }
      return true;
    }
    if (S >= std::max(nt[0], nt[1])) return false;
  }
}

// The Q route's contractions may run in FP32 (under chol_prec FP32) only while
// the quadratic form is short: it sums M^2 N^2 terms of both signs per spin,
// and the FP32 rounding error grows with their number (measured per-step E_L
// error: within 0.1 mHa at M N = 1250, 2.2e-4 Ha at M N = 10000).  Above
// the limit the Q route runs FP64 in every mode.
bool q_fp32_ok(int M, int n_up, int n_dn) {
  return (long)M * std::max(n_up, n_dn) <= AFQMC_QROUTE_FP32_MAX_K;
}

bool use_qroute(int M, int G, int n_up, int n_dn, int n_det) {
  if (n_det != 1 || G < 2 * M) return false;
  if ((long)M * std::max(n_up, n_dn) > 16384) return false;
  int ns[2];
  return q_plan(M, G, n_up, n_dn, nullptr, ns);
}

// Elements of the exchange kernels' repacked A operand for one spin (NP <= 64).
size_t pack_exchange_elems(size_t G, size_t MP4, size_t NP) {
  const size_t KB = (MP4 / 4 + 3) / 4;
  return G * KB * 64 * 4 * (NP / 16);
}

afq::SpinGeom spin_geom(const afqmc_trial* tr, int s, afqmc_prec prec) {
  const bool fp32 = prec == AFQMC_FP32;
  afq::SpinGeom g;
  g.N = tr->nel[s];
  g.off = s ? tr->nel[0] : 0;
  g.NP = tr->NP[s];
  g.C = tr->C[s];
  g.htil = tr->htil[s];
  g.Lt = (prec == AFQMC_BF16 || prec == AFQMC_BF16X3) ? tr->Ltbf[s]
         : fp32 ? (const void*)tr->Lt32[s] : (const void*)tr->Lt64[s];
  g.Apk = fp32 ? (const void*)tr->Apk32[s] : (const void*)tr->Apk64[s];
  return g;
}

afq::MDParams md_params(const afqmc_trial* tr, bool fp32) {
  afq::MDParams p;
  p.M = tr->ham->M;
  p.Nt = tr->Nt;
  p.G = tr->ham->G;
  p.n_det = tr->n_det;
  p.MP4 = tr->MP4;
  p.e_core = tr->ham->e_core;
  for (int s = 0; s < 2; ++s) {
    p.sp[s].N = tr->nel[s];
    p.sp[s].off = s ? tr->nel[0] : 0;
    p.sp[s].C = tr->C[s];
    p.sp[s].LC = fp32 ? (const void*)tr->LC32[s] : (const void*)tr->LC64[s];
  }
  p.exc = tr->d_exc;
  p.coeff = tr->d_coeff;
  std::memset(&p.rows, 0, sizeof(p.rows));
  if (fp32 && tr->md_rows) {
    p.rows.ok = 1;
    p.rows.KS = tr->mdKS;
    for (int s = 0; s < 2; ++s) {
      p.rows.R[s] = tr->mdR[s];
      p.rows.RP[s] = tr->mdRP[s];
      p.rows.npair[s] = tr->mdnp[s];
      p.rows.LCc[s] = tr->LCc[s];
      p.rows.pair[s] = tr->d_mdpair[s];
      p.rows.pbeg[s] = tr->d_mdpbeg[s];
    }
    p.rows.dx = tr->d_mddx;
  }
  return p;
}

// Theta as the FP64 matrix in ws.th_*, or as the Q route's split rows in
// ws.P_* (contraction type).
afq::ThetaOut fp64_out(const WS& ws) {
  afq::ThetaOut o;
  o.thr = ws.th_re;
  o.thi = ws.th_im;
  return o;
}

afq::ThetaOut split_out(const afqmc_trial* tr, const WS& ws, bool f32) {
  afq::ThetaOut o;
  o.sr = ws.P_re;
  o.si = ws.P_im;
  o.Ktot = tr->Kp[0] + tr->Kp[1];
  o.Kp0 = tr->Kp[0];
  o.f32 = f32;
  return o;
}

// Overlap / Theta / exchange / combination for the current phi; leaves the new
// log overlap and E_L in ws.lsn / ws.eln and the force-bias traces in ws.v.
afqmc_status measure_qroute(afqmc_trial* tr, afqmc_walkers* wk, const WS& ws, bool fp32,
                            hipStream_t st);

afqmc_status measure_core(afqmc_trial* tr, afqmc_walkers* wk, const WS& ws, afqmc_prec chol,
                          hipStream_t st) {
  afqmc_ham* hm = tr->ham;
  const int W = wk->n_walkers, M = hm->M, G = hm->G, Nt = tr->Nt;
  const bool f32 = chol == AFQMC_FP32;
  const afq::SpinGeom s0 = spin_geom(tr, 0, chol), s1 = spin_geom(tr, 1, chol);
  const bool bf = chol == AFQMC_BF16 || chol == AFQMC_BF16X3;
  const bool qr = tr->n_det == 1 && G > 0 && tr->qroute && !bf;
  const bool q32 = f32 && tr->q32;  // Q-route contraction type
  {
    TimedLaunch tl(&hm->timer, KC_OVERLAP, st);
    AFQ_CK(afq::overlap_theta(st, W, M, Nt, s0, s1, wk->phi_re, wk->phi_im,
                              qr ? split_out(tr, ws, q32) : fp64_out(ws), ws.ld_re, ws.ld_im,
                              ws.e1_re, ws.e1_im, hm->max_lds));
  }
  if (tr->n_det > 1) {
    const afq::MDParams mp = md_params(tr, f32);
    {
      TimedLaunch tl(&hm->timer, KC_OTHER, st);
      AFQ_CK(afq::md_overlap(st, W, mp, ws.th_re, ws.th_im, ws.ld_re, ws.ld_im, ws.c0_re, ws.c0_im,
                             ws.tot_re, ws.tot_im, ws.lsn_re, ws.lsn_im, hm->max_lds));
    }
    TimedLaunch tl(&hm->timer, KC_EXCHANGE, st);
    if (f32) {
      AFQ_CK(afq::md_energy<float>(st, W, mp, ws.th_re, ws.th_im, ws.c0_re, ws.c0_im, ws.tot_re,
                                   ws.tot_im, ws.v_re, ws.v_im, ws.eln_re, ws.eln_im, ws.vfin,
                                   hm->max_lds));
    } else {
      AFQ_CK(afq::md_energy<double>(st, W, mp, ws.th_re, ws.th_im, ws.c0_re, ws.c0_im, ws.tot_re,
                                    ws.tot_im, ws.v_re, ws.v_im, ws.eln_re, ws.eln_im, ws.vfin,
                                    hm->max_lds));
    }
    return AFQMC_OK;
  }
  if (qr) return measure_qroute(tr, wk, ws, q32, st);
  if (G > 0) {
    TimedLaunch tl(&hm->timer, KC_EXCHANGE, st);
    if (bf) {
      const bool x3 = chol == AFQMC_BF16X3;
      AFQ_CK(afq::exchange_bf16(st, W, M, tr->MP32, Nt, G, s0, s1, x3 ? tr->Ltbf_lo[0] : nullptr,
                                x3 ? tr->Ltbf_lo[1] : nullptr, ws.th_re, ws.th_im, ws.vs_re,
                                ws.vs_im, ws.exx_re, ws.exx_im, hm->max_lds));
    } else if (f32) {
      AFQ_CK(afq::exchange<float>(st, W, M, tr->MP4, Nt, G, s0, s1, ws.th_re, ws.th_im, ws.vs_re,
                                  ws.vs_im, ws.exx_re, ws.exx_im, hm->max_lds));
    } else {
      AFQ_CK(afq::exchange<double>(st, W, M, tr->MP4, Nt, G, s0, s1, ws.th_re, ws.th_im, ws.vs_re,
                                   ws.vs_im, ws.exx_re, ws.exx_im, hm->max_lds));
    }
  } else {
    AFQ_CK(hipMemsetAsync(ws.exx_re, 0, 2 * W * sizeof(double), st));
    AFQ_CK(hipMemsetAsync(ws.exx_im, 0, 2 * W * sizeof(double), st));
  }
  AFQ_CK(afq::combine_single(st, W, G, hm->e_core, ws.vs_re, ws.vs_im, ws.exx_re, ws.exx_im,
                             ws.e1_re, ws.e1_im, ws.ld_re, ws.ld_im, ws.v_re, ws.v_im, ws.lsn_re,
                             ws.lsn_im, ws.eln_re, ws.eln_im, ws.vfin));
  return AFQMC_OK;
}

afqmc_status measure_set(afqmc_trial* tr, afqmc_walkers* wk, const WS& ws, afqmc_prec chol,
                         hipStream_t st) {
  afqmc_status s = measure_core(tr, wk, ws, chol, st);
  if (s != AFQMC_OK) return s;
  AFQ_CK(afq::weight_update(st, wk->n_walkers, 0, 0.0, 0.0, ws.lsn_re, ws.lsn_im, ws.eln_re,
                            ws.eln_im, ws.mf_re, ws.mf_im, ws.vfin, wk->weight, wk->logovlp_re,
                            wk->logovlp_im, wk->eloc_re, wk->eloc_im, ws.dead));
  return AFQMC_OK;
}

afqmc_status orthonormalize_impl(afqmc_trial* tr, afqmc_walkers* wk, const WS& ws, hipStream_t st) {
  afqmc_ham* hm = tr->ham;
  const int W = wk->n_walkers;
  {
    TimedLaunch tl(&hm->timer, KC_MGS, st);
    AFQ_CK(afq::mgs(st, W, hm->M, tr->Nt, tr->nel[0], tr->nel[1], wk->phi_re, wk->phi_im,
                    hm->max_lds));
  }
  const afq::SpinGeom s0 = spin_geom(tr, 0, AFQMC_FP64), s1 = spin_geom(tr, 1, AFQMC_FP64);
  // log det and E1 only: Theta is not stored (multi-determinant trials need it)
  AFQ_CK(afq::overlap_theta(st, W, hm->M, tr->Nt, s0, s1, wk->phi_re, wk->phi_im,
                            tr->n_det > 1 ? fp64_out(ws) : afq::ThetaOut(), ws.ld_re, ws.ld_im,
                            ws.e1_re, ws.e1_im, hm->max_lds));
  if (tr->n_det > 1) {
    const afq::MDParams mp = md_params(tr, false);
    AFQ_CK(afq::md_overlap(st, W, mp, ws.th_re, ws.th_im, ws.ld_re, ws.ld_im, ws.c0_re, ws.c0_im,
                           ws.tot_re, ws.tot_im, ws.lsn_re, ws.lsn_im, hm->max_lds));
  } else {
  // log S = sum over spins of log det (single determinant)
  AFQ_CK(afq::combine_single(st, W, 0, 0.0, ws.vs_re, ws.vs_im, ws.exx_re, ws.exx_im, ws.e1_re,
                             ws.e1_im, ws.ld_re, ws.ld_im, ws.v_re, ws.v_im, ws.lsn_re,
                             ws.lsn_im, ws.eln_re, ws.eln_im, ws.vfin));
  }
  AFQ_CK(afq::weight_update(st, W, 2, 0.0, 0.0, ws.lsn_re, ws.lsn_im, ws.eln_re, ws.eln_im,
                            ws.mf_re, ws.mf_im, ws.vfin, wk->weight, wk->logovlp_re,
                            wk->logovlp_im, wk->eloc_re, wk->eloc_im, ws.dead));
  return AFQMC_OK;
}

afqmc_status reconfigure_impl(afqmc_trial* tr, afqmc_walkers* wk, const WS& ws, uint64_t seed,
                              uint64_t pc_index, hipStream_t st) {
  afqmc_ham* hm = tr->ham;
  const int W = wk->n_walkers;
  const long row = (long)hm->M * tr->Nt, G = hm->G;
  {
    TimedLaunch tl(&hm->timer, KC_COMB, st);
    AFQ_CK(afq::comb_parents(st, W, wk->weight, seed, pc_index, wk->system_id, ws.cbuf, ws.parent,
                             ws.scal + 2));
  }
  double* snap = ws.snap;
  struct Item { double* p; long row; };
  const Item items[] = {{wk->phi_re, row},     {wk->phi_im, row},     {wk->logovlp_re, 1},
                        {wk->logovlp_im, 1},   {wk->eloc_re, 1},      {wk->eloc_im, 1},
                        {ws.v_re, G},          {ws.v_im, G}};
  for (const Item& it : items) {
    if (it.row == 0) continue;
    AFQ_CK(hipMemcpyAsync(snap, it.p, (size_t)W * it.row * sizeof(double), hipMemcpyDeviceToDevice, st));
    AFQ_CK(afq::gather_rows(st, W, it.row, ws.parent, snap, it.p));
    snap += (size_t)W * it.row;
  }
  AFQ_CK(afq::comb_weights(st, W, ws.scal + 2, wk->weight));
  return AFQMC_OK;
}

B1Entry* get_b1(afqmc_trial* tr, double dt, hipStream_t st, afqmc_status* err) {
  for (auto& e : tr->b1)
    if (e.dt == dt) return &e;
  const int M = tr->ham->M;
  std::vector<double> V, lam;
  jacobi_eigh(M, tr->H1p, V, lam);
  B1Entry e;
  e.dt = dt;
  e.h64.assign((size_t)M * M, 0.0);
  // B1 - I = V diag(expm1(-dt lam / 2)) V^T
  for (int i = 0; i < M; ++i)
    for (int j = 0; j < M; ++j) {
      double s = 0.0;
      for (int k = 0; k < M; ++k) s += V[(size_t)i * M + k] * std::expm1(-0.5 * dt * lam[k]) * V[(size_t)j * M + k];
      e.h64[(size_t)i * M + j] = s;
    }
  e.h32.resize(e.h64.size());
  for (size_t i = 0; i < e.h64.size(); ++i) e.h32[i] = (float)e.h64[i];
  void* p64 = nullptr;
  void* p32 = nullptr;
  if (tr->arena.alloc(&p64, e.h64.size() * sizeof(double)) != hipSuccess ||
      tr->arena.alloc(&p32, e.h32.size() * sizeof(float)) != hipSuccess) {
    *err = fail(AFQMC_ERR_OOM, "B1 allocation failed");
    return nullptr;
  }
  e.d64 = (double*)p64;
  e.d32 = (float*)p32;
  if (hipMemcpy(e.d64, e.h64.data(), e.h64.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(e.d32, e.h32.data(), e.h32.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
    *err = fail(AFQMC_ERR_DEVICE, "B1 upload failed");
    return nullptr;
  }
  (void)st;
  tr->b1.push_back(std::move(e));
  return &tr->b1.back();
}

struct Bf16Tag {};

// Force bias v_g = sum_k ts[k] Lq[k][g] for all walkers (single determinant)
// from the split Theta rows in ws.P_* (contraction type), as a GEMM split over
// k into nz partials in ws.ACC_* (free outside the propagation; float
// partials when the contraction is FP32, as the MFMA accumulated them);
// returns nz.
int force_bias_partials(afqmc_trial* tr, afqmc_walkers* wk, const WS& ws, bool fp32,
                        hipStream_t st, hipError_t* err) {
  afqmc_ham* hm = tr->ham;
  const int W = wk->n_walkers, M = hm->M, G = hm->G, Nt = tr->Nt;
  const int Ktot = tr->Kp[0] + tr->Kp[1];
  const int nz = afq::fbias_nz(W, Ktot, G, acc_cap(M, G, Nt));
  if (fp32)
    *err = afq::fbias_mm<float>(st, W, Ktot, G, tr->Gp, nz, (const float*)ws.P_re,
                                (const float*)ws.P_im, tr->Lq32, (float*)ws.ACC_re,
                                (float*)ws.ACC_im);
  else
    *err = afq::fbias_mm<double>(st, W, Ktot, G, tr->Gp, nz, ws.P_re, ws.P_im, tr->Lq64, ws.ACC_re,
                                 ws.ACC_im);
  return nz;
}

// E_L by the Q route (single determinant) from the split Theta rows in
// ws.P_*: force-bias partials (ws.ACC_*), theta^T Q theta segment partials
// (ws.Ta_re), then one combination kernel for v, exx, E_L and log S.
afqmc_status measure_qroute(afqmc_trial* tr, afqmc_walkers* wk, const WS& ws, bool fp32,
                            hipStream_t st) {
  afqmc_ham* hm = tr->ham;
  const int W = wk->n_walkers, G = hm->G;
  int nz;
  {
    TimedLaunch tl(&hm->timer, KC_FBIAS, st);
    hipError_t e;
    nz = force_bias_partials(tr, wk, ws, fp32, st, &e);
    AFQ_CK(e);
  }
  const int nseg = tr->nseg[0] + tr->nseg[1];
  double* qpart = (double*)ws.Ta_re;
  {
    TimedLaunch tl(&hm->timer, KC_EXCHANGE, st);
    if (fp32) {
      AFQ_CK(afq::qform<float>(st, W, tr->Kp[0], tr->Kp[1], nseg, tr->qsegs, (const float*)ws.P_re,
                               (const float*)ws.P_im, tr->Q32[0], tr->Q32[1], qpart));
    } else {
      AFQ_CK(afq::qform<double>(st, W, tr->Kp[0], tr->Kp[1], nseg, tr->qsegs, ws.P_re, ws.P_im,
                                tr->Q64[0], tr->Q64[1], qpart));
    }
  }
  TimedLaunch tl(&hm->timer, KC_OTHER, st);
  if (fp32)
    AFQ_CK(afq::combine_qroute<float>(st, W, G, nz, tr->nseg[0], tr->nseg[1], hm->e_core,
                                      (const float*)ws.ACC_re, (const float*)ws.ACC_im, qpart,
                                      ws.e1_re, ws.e1_im, ws.ld_re, ws.ld_im, ws.v_re, ws.v_im,
                                      ws.exx_re, ws.exx_im, ws.lsn_re, ws.lsn_im, ws.eln_re,
                                      ws.eln_im, ws.vfin));
  else
    AFQ_CK(afq::combine_qroute<double>(st, W, G, nz, tr->nseg[0], tr->nseg[1], hm->e_core,
                                       ws.ACC_re, ws.ACC_im, qpart, ws.e1_re, ws.e1_im, ws.ld_re,
                                       ws.ld_im, ws.v_re, ws.v_im, ws.exx_re, ws.exx_im,
                                       ws.lsn_re, ws.lsn_im, ws.eln_re, ws.eln_im, ws.vfin));
  return AFQMC_OK;
}

afqmc_status hybrid_force_bias(afqmc_trial* tr, afqmc_walkers* wk, const WS& ws, bool fp32,
                               hipStream_t st) {
  afqmc_ham* hm = tr->ham;
  const int W = wk->n_walkers, M = hm->M, G = hm->G, Nt = tr->Nt;
  const afq::SpinGeom s0 = spin_geom(tr, 0, AFQMC_FP64), s1 = spin_geom(tr, 1, AFQMC_FP64);
  {
    TimedLaunch tl(&hm->timer, KC_OVERLAP, st);
    AFQ_CK(afq::overlap_theta(st, W, M, Nt, s0, s1, wk->phi_re, wk->phi_im,
                              split_out(tr, ws, fp32), ws.ld_re, ws.ld_im, ws.e1_re, ws.e1_im,
                              hm->max_lds));
  }
  int nz;
  {
    TimedLaunch tl(&hm->timer, KC_FBIAS, st);
    hipError_t e;
    nz = force_bias_partials(tr, wk, ws, fp32, st, &e);
    AFQ_CK(e);
  }
  if (fp32)
    AFQ_CK(afq::hybrid_force_bias_finish<float>(st, W, G, nz, (const float*)ws.ACC_re,
                                                (const float*)ws.ACC_im, ws.v_re, ws.v_im,
                                                ws.ld_re, ws.ld_im, ws.lsn_re, ws.lsn_im,
                                                ws.vfin));
  else
    AFQ_CK(afq::hybrid_force_bias_finish<double>(st, W, G, nz, ws.ACC_re, ws.ACC_im, ws.v_re,
                                                 ws.v_im, ws.ld_re, ws.ld_im, ws.lsn_re,
                                                 ws.lsn_im, ws.vfin));
  return AFQMC_OK;
}

template <typename TC, typename TT>
afqmc_status propagate_typed(afqmc_trial* tr, afqmc_walkers* wk, const WS& ws, B1Entry* b1,
                             int n_steps, double dt, uint64_t seed, uint64_t step0,
                             const afqmc_options* opt, double* emix_dev, hipStream_t st) {
  afqmc_ham* hm = tr->ham;
  const int W = wk->n_walkers, M = hm->M, G = hm->G, Nt = tr->Nt;
  const long mn = (long)M * Nt, mm = (long)M * M;
  const TC* Lc = std::is_same<TC, float>::value ? (const TC*)hm->Lf : (const TC*)hm->L;
  const TC* Lpc = std::is_same<TC, float>::value ? (const TC*)hm->Lpf : (const TC*)hm->Lp;
  const int Mp = M * (M + 1) / 2;
  constexpr bool BF = std::is_same<TC, Bf16Tag>::value;
  const TT* B1m = std::is_same<TT, float>::value ? (const TT*)b1->d32 : (const TT*)b1->d64;
  TC* coefT = (TC*)ws.coefT;  // [2W][Gp] row-major (BF16: the kernels' own layout)
  const int Gp = (G + 63) / 64 * 64;
  TT* A = (TT*)ws.A;
  TT* Tbuf[2][2] = {{(TT*)ws.Ta_re, (TT*)ws.Ta_im}, {(TT*)ws.Tb_re, (TT*)ws.Tb_im}};
  const bool hybrid = opt->weight_mode == AFQMC_WEIGHT_HYBRID;
  double* hyr = hybrid ? ws.hy_re : nullptr;
  double* hyi = hybrid ? ws.hy_im : nullptr;
  for (int s = 0; s < n_steps; ++s) {
    const uint64_t t = step0 + (uint64_t)s;
    const bool measuring = !hybrid || (t + 1) % (uint64_t)opt->meas_every == 0;
    // BF16X3: the coefficients' second terms follow the first ones in coefT
    const bool x3 = opt->chol_prec == AFQMC_BF16X3;
    void* coef_lo = x3 ? (void*)((char*)ws.coefT + (size_t)2 * W * G * 2) : nullptr;
    if constexpr (BF) {
      AFQ_CK(afq::fields_coeff_bf16(st, W, G, G, seed, t, wk->system_id, dt, ws.v_re, ws.v_im,
                                    tr->lbar, ws.coefT, coef_lo, ws.mf_re, ws.mf_im, hyr, hyi));
    } else {
      AFQ_CK(afq::fields_coeff<TC>(st, W, G, Gp, seed, t, wk->system_id, dt, ws.v_re, ws.v_im,
                                   tr->lbar, coefT, ws.mf_re, ws.mf_im, nullptr, hyr, hyi));
    }
    const bool fused = afq::propagate_fused_fits(M, Nt, sizeof(TT), hm->max_lds);
    const bool packed = fused && !BF;  // A as upper triangles (A is symmetric)
    if (G > 0) {
      TimedLaunch tl(&hm->timer, KC_ABUILD, st);
      if constexpr (BF) {
        AFQ_CK(afq::gemm_bf16<TT>(st, 2 * W, (int)mm, G, ws.coefT, coef_lo, G, hm->Lbf,
                                  x3 ? hm->Lbf_lo : nullptr, (int)mm, A, (int)mm, 1.0));
      } else if (packed) {
        AFQ_CK((afq::abuild<TC, TT>(st, 2 * W, Mp, G, Gp, coefT, Lpc, A)));
      } else {
        AFQ_CK((afq::abuild<TC, TT>(st, 2 * W, (int)mm, G, Gp, coefT, Lc, A)));
      }
    } else {
      AFQ_CK(hipMemsetAsync(A, 0, (size_t)W * 2 * mm * sizeof(TT), st));
    }
    // phi -> P = B1 phi, ACC = P
    {
    TimedLaunch tl_t(&hm->timer, KC_TAYLOR, st);
    if (fused) {
      AFQ_CK(afq::propagate_fused<TT>(st, W, M, Nt, opt->taylor_order, packed, A, B1m, wk->phi_re,
                                      wk->phi_im, hm->max_lds));
    } else {
    AFQ_CK((afq::cgemm_walkers<TT, double, false, 0>(st, W, M, Nt, M, B1m, nullptr, M, 0,
                                                     wk->phi_re, wk->phi_im, Nt, mn, nullptr,
                                                     nullptr, ws.P_re, ws.P_im, ws.ACC_re,
                                                     ws.ACC_im, Nt, mn, 1.0)));
    // Taylor terms T_n = A T_{n-1} / n, ACC += T_n
    for (int n = 1; n <= opt->taylor_order; ++n) {
      TT* outr = Tbuf[(n - 1) & 1][0];
      TT* outi = Tbuf[(n - 1) & 1][1];
      if (n == 1) {
        AFQ_CK((afq::cgemm_walkers<TT, double, true, 1>(st, W, M, Nt, M, A, A + mm, M, 2 * mm,
                                                        ws.P_re, ws.P_im, Nt, mn, outr, outi,
                                                        ws.ACC_re, ws.ACC_im, nullptr, nullptr, Nt,
                                                        mn, 1.0)));
      } else {
        const TT* inr = Tbuf[n & 1][0];
        const TT* ini = Tbuf[n & 1][1];
        AFQ_CK((afq::cgemm_walkers<TT, TT, true, 1>(st, W, M, Nt, M, A, A + mm, M, 2 * mm, inr, ini,
                                                    Nt, mn, outr, outi, ws.ACC_re, ws.ACC_im,
                                                    nullptr, nullptr, Nt, mn, 1.0 / n)));
      }
    }
    // phi = ACC + (B1 - I) ACC
    AFQ_CK((afq::cgemm_walkers<TT, double, false, 0>(st, W, M, Nt, M, B1m, nullptr, M, 0,
                                                     ws.ACC_re, ws.ACC_im, Nt, mn, nullptr,
                                                     nullptr, wk->phi_re, wk->phi_im, nullptr,
                                                     nullptr, Nt, mn, 1.0)));
    }
    }
    afqmc_status rs;
    if (hybrid && !measuring && tr->n_det == 1 && G > 0)
      rs = hybrid_force_bias(tr, wk, ws, opt->chol_prec != AFQMC_FP64 && tr->q32, st);
    else
      rs = measure_core(tr, wk, ws, opt->chol_prec, st);
    if (rs != AFQMC_OK) return rs;
    AFQ_CK(afq::weight_update(st, W, hybrid ? (measuring ? 3 : 4) : 1, dt, opt->e_trial, ws.lsn_re,
                              ws.lsn_im, ws.eln_re, ws.eln_im, ws.mf_re, ws.mf_im, ws.vfin,
                              wk->weight, wk->logovlp_re, wk->logovlp_im, wk->eloc_re, wk->eloc_im,
                              ws.dead, ws.hy_re, ws.hy_im, tr->e0_shift));
    AFQ_CK(afq::reset_dead(st, W, M, Nt, G, ws.dead, tr->D0, tr->ref_ls[0], tr->ref_ls[1],
                           tr->ref_el[0], tr->ref_el[1], tr->vref_re, tr->vref_im, wk->phi_re,
                           wk->phi_im, wk->logovlp_re, wk->logovlp_im, wk->eloc_re, wk->eloc_im,
                           ws.v_re, ws.v_im));
    if (measuring) {
      AFQ_CK(afq::mixed_energy(st, W, wk->weight, wk->eloc_re, emix_dev ? emix_dev + s : ws.scal,
                               ws.scal + 1));
    } else if (emix_dev) {
      AFQ_CK(afq::fill(st, emix_dev + s, 1, std::numeric_limits<double>::quiet_NaN()));
    }
    if (opt->ortho_every > 0 && (t + 1) % (uint64_t)opt->ortho_every == 0) {
      rs = orthonormalize_impl(tr, wk, ws, st);
      if (rs != AFQMC_OK) return rs;
    }
    if (opt->pc_every > 0 && (t + 1) % (uint64_t)opt->pc_every == 0) {
      rs = reconfigure_impl(tr, wk, ws, seed, t, st);
      if (rs != AFQMC_OK) return rs;
    }
  }
  return AFQMC_OK;
}

}  // namespace

namespace afq {
// The thread's last-error message, for the ABI functions of other files.
afqmc_status set_error(afqmc_status s, const char* msg) { return fail(s, msg); }

// The comb of afqmc_reconfigure with its scratch (prefix sums, parents, norm
// factor, gather snapshot) carved from the device buffer `scratch` of
// `scratch_bytes` instead of the walker workspace; the workspace still holds
// the walkers' force-bias traces, which are gathered with the rest.  The
// snapshot is used column range by column range, so any walker shape fits
// once the parents, prefix sums and one column of all walkers do.  Enqueues
// nothing that allocates.
afqmc_status reconfigure_scratch(afqmc_trial* tr, afqmc_walkers* wk, uint64_t seed,
                                 uint64_t pc_index, char* scratch, size_t scratch_bytes,
                                 double* norm_factor_host, hipStream_t st) {
  if (!tr) return fail(AFQMC_ERR_ARG, "NULL trial");
  afqmc_status s = check_walkers(tr, wk);
  if (s != AFQMC_OK) return s;
  const int W = wk->n_walkers;
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t head = 256 + up((size_t)W * sizeof(int)) + up((size_t)W * sizeof(double));
  if (!scratch || scratch_bytes < head + (size_t)W * sizeof(double))
    return fail(AFQMC_ERR_ARG, "n_walkers too large for the scratch buffer");
  double* norm = (double*)scratch;
  int* parent = (int*)(scratch + 256);
  double* cbuf = (double*)(scratch + 256 + up((size_t)W * sizeof(int)));
  double* snap = (double*)(scratch + head);
  const size_t snap_doubles = (scratch_bytes - head) / sizeof(double);
  afqmc_ham* hm = tr->ham;
  AFQ_CK(hipSetDevice(hm->device));
  const WS ws = layout(tr, W, wk->workspace);
  const long row = (long)hm->M * tr->Nt, G = hm->G;
  // (no kernel timing here: its events may be created on demand)
  AFQ_CK(afq::comb_parents(st, W, wk->weight, seed, pc_index, wk->system_id, cbuf, parent, norm));
  struct Item { double* p; long row; };
  const Item items[] = {{wk->phi_re, row},     {wk->phi_im, row},     {wk->logovlp_re, 1},
                        {wk->logovlp_im, 1},   {wk->eloc_re, 1},      {wk->eloc_im, 1},
                        {ws.v_re, G},          {ws.v_im, G}};
  for (const Item& it : items)
    AFQ_CK(afq::gather_rows_chunked(st, W, it.row, parent, it.p, snap, snap_doubles));
  AFQ_CK(afq::comb_weights(st, W, norm, wk->weight));
  if (norm_factor_host) {
    AFQ_CK(hipMemcpyAsync(norm_factor_host, norm, sizeof(double), hipMemcpyDeviceToHost, st));
    AFQ_CK(hipStreamSynchronize(st));
    if (!(*norm_factor_host > 0.0))
      return fail(AFQMC_ERR_NONFINITE, "comb: the sum of weights is not positive and finite");
  }
  return AFQMC_OK;
}

// Device of a trial (for callers outside this file).
int trial_device(const afqmc_trial* tr) { return tr->ham->device; }
}  // namespace afq

extern "C" {

const char* afqmc_last_error(void) { return g_err.c_str(); }

afqmc_status afqmc_init_hamiltonian(afqmc_ham** out, int device, void* stream, int M, int n_chol,
                                    const double* h, const double* L, double e_core) {
  if (!out) return fail(AFQMC_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (M < 1 || M > AFQMC_MAX_M) return fail(AFQMC_ERR_ARG, "M must be in [1, AFQMC_MAX_M]");
  if (n_chol < 0) return fail(AFQMC_ERR_ARG, "n_chol must be >= 0");
  if (!h) return fail(AFQMC_ERR_ARG, "h is NULL");
  if (n_chol > 0 && !L) return fail(AFQMC_ERR_ARG, "L is NULL");
  if (!std::isfinite(e_core)) return fail(AFQMC_ERR_ARG, "e_core is not finite");
  if (!all_finite(h, (size_t)M * M) || (n_chol > 0 && !all_finite(L, (size_t)n_chol * M * M)))
    return fail(AFQMC_ERR_ARG, "h or L has a non-finite entry");
  if (!symmetric(h, M, 1e-10)) return fail(AFQMC_ERR_ARG, "h is not symmetric");
  for (int g = 0; g < n_chol; ++g)
    if (!symmetric(L + (size_t)g * M * M, M, 1e-10))
      return fail(AFQMC_ERR_ARG, "L[" + std::to_string(g) + "] is not symmetric");
  int ndev = 0;
  AFQ_CK(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(AFQMC_ERR_ARG, "no such device");
  AFQ_CK(hipSetDevice(device));
  hipStream_t st = (hipStream_t)stream;
  afqmc_ham* hm = new afqmc_ham();
  hm->device = device;
  hm->M = M;
  hm->G = n_chol;
  hm->e_core = e_core;
  hm->h_host.assign(h, h + (size_t)M * M);
  int lds = 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess && lds > 0)
    hm->max_lds = (size_t)lds;
  const size_t mm = (size_t)M * M, gmm = (size_t)n_chol * mm;
  void *ph, *pL, *pLf, *pL2, *pLb;
  if (hm->arena.alloc(&ph, mm * 8) || hm->arena.alloc(&pL, gmm * 8) ||
      hm->arena.alloc(&pLf, gmm * 4) || hm->arena.alloc(&pL2, mm * 8) ||
      hm->arena.alloc(&pLb, gmm * 2) || hm->arena.alloc(&hm->Lbf_lo, gmm * 2) ||
      hm->arena.alloc((void**)&hm->Lp, (size_t)n_chol * (mm + M) / 2 * 8) ||
      hm->arena.alloc((void**)&hm->Lpf, (size_t)n_chol * (mm + M) / 2 * 4)) {
    hm->arena.release();
    delete hm;
    return fail(AFQMC_ERR_OOM, "hamiltonian allocation failed");
  }
  hm->h = (double*)ph;
  hm->L = (double*)pL;
  hm->Lf = (float*)pLf;
  hm->L2 = (double*)pL2;
  hm->Lbf = pLb;
  auto bad = [&](const char* what) {
    hm->arena.release();
    delete hm;
    return fail(AFQMC_ERR_DEVICE, what);
  };
  if (hipMemcpyAsync(hm->h, h, mm * 8, hipMemcpyHostToDevice, st) != hipSuccess) return bad("h upload");
  if (n_chol > 0) {
    if (hipMemcpyAsync(hm->L, L, gmm * 8, hipMemcpyHostToDevice, st) != hipSuccess) return bad("L upload");
    if (afq::convert_f64_f32(st, hm->L, hm->Lf, (long)gmm) != hipSuccess) return bad("L convert");
    {  // upper triangles, row by row
      std::vector<double> lp((size_t)n_chol * (mm + M) / 2);
      size_t o = 0;
      for (int g = 0; g < n_chol; ++g)
        for (int i = 0; i < M; ++i)
          for (int j = i; j < M; ++j) lp[o++] = L[(size_t)g * mm + (size_t)i * M + j];
      if (hipMemcpyAsync(hm->Lp, lp.data(), lp.size() * 8, hipMemcpyHostToDevice, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess ||
          afq::convert_f64_f32(st, hm->Lp, hm->Lpf, (long)lp.size()) != hipSuccess)
        return bad("packed L");
    }
    if (afq::convert_f64_bf16(st, hm->L, hm->Lbf, (long)gmm) != hipSuccess ||
        afq::convert_f64_bf16_lo(st, hm->L, hm->Lbf_lo, (long)gmm) != hipSuccess)
      return bad("L convert");
  }
  // sum_g L_g L_g as one GEMM over the stacked index (g, k)
  if (afq::gemm_real<double, double, true>(st, M, M, n_chol * M, hm->L, M, 0, hm->L, M, 0, hm->L2,
                                           M, 0, 1, 1.0) != hipSuccess)
    return bad("sum L^2");
  if (hipStreamSynchronize(st) != hipSuccess) return bad("init sync");
  *out = hm;
  return AFQMC_OK;
}

void afqmc_free_hamiltonian(afqmc_ham* hm) {
  if (!hm) return;
  (void)hipSetDevice(hm->device);
  hm->arena.release();
  delete hm;
}

namespace {

// Whether the compact-row FP32 energy kernel's limits admit a multi-determinant
// trial of these sizes (its tables are then built at set-up).
bool md_rows_sizes_ok(int M, int n_up, int n_dn, int n_det) {
  return n_det > 1 && M <= afq::kMdRowsMaxM && n_det <= afq::kMdRowsMaxDet &&
         n_up <= afq::kMdRowsMaxN && n_dn <= afq::kMdRowsMaxN;
}

// Upper bound of the compact-row tables' bytes (rows: N + the distinct
// particles, at most 2 (n_det - 1) of them), counted by the footprint.
size_t md_rows_bound_bytes(int M, int G, int n_up, int n_dn, int n_det) {
  if (!md_rows_sizes_ok(M, n_up, n_dn, n_det)) return 0;
  auto rnd = [](size_t b) { return (std::max<size_t>(b, 256) + 255) / 256 * 256; };
  const int nel[2] = {n_up, n_dn};
  size_t t = rnd((size_t)n_det * afq::kMdDx * 4);
  for (int s = 0; s < 2; ++s) {
    if (!nel[s]) continue;
    const size_t rp = round_up(std::min(M, nel[s] + 2 * (n_det - 1)), 16);
    const size_t rows = M <= 64 ? 64 : 128;  // 4 KS
    t += rnd((size_t)(G + 2) * rows * rp * 4) + rnd((size_t)n_det * 16) + 2 * rnd((size_t)M * 4);
  }
  return t;
}

// Per spin: the rows the determinants read (the N occupied orbitals, then
// the distinct particle orbitals ascending), the distinct (particle, hole)
// pairs, and the packed per-determinant words; then LCc = those rows of LC
// (slots 0..G) and of C (slot G+1) in FP32.  Leaves md_rows false (the FP32
// energy runs the full-row kernel) when a limit is not met.
afqmc_status md_rows_setup(afqmc_trial* tr, const std::vector<int>& exc, hipStream_t st) {
  const int M = tr->ham->M, G = tr->ham->G, n_det = tr->n_det;
  tr->md_rows = false;
  if (!md_rows_sizes_ok(M, tr->nel[0], tr->nel[1], n_det)) return AFQMC_OK;
  // slot order of the determinants: by the larger excitation rank of the two
  // spins, then by the ranks, so that the 64-lane slots mix few ranks per spin
  std::vector<int> order(n_det);
  for (int i = 0; i < n_det; ++i) order[i] = i;
  auto rank = [&](int i, int s) { return exc[((size_t)i * 2 + s) * 5]; };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    const int ka[3] = {std::max(rank(a, 0), rank(a, 1)), rank(a, 0), rank(a, 1)};
    const int kb[3] = {std::max(rank(b, 0), rank(b, 1)), rank(b, 0), rank(b, 1)};
    return std::lexicographical_compare(ka, ka + 3, kb, kb + 3);
  });
  std::vector<int> dx((size_t)n_det * afq::kMdDx, 0), rowmap[2], pairs[2], pbeg[2];
  for (int k = 0; k < n_det; ++k) dx[(size_t)k * afq::kMdDx + 6] = order[k];
  int R[2], RP[2];
  const int KS = M <= 64 ? 16 : 32;  // k steps: 4 KS >= M rows
  for (int s = 0; s < 2; ++s) {
    const int N = tr->nel[s];
    std::vector<int> vl;
    for (int i = 0; i < n_det; ++i) {
      const int* d = &exc[((size_t)i * 2 + s) * 5];
      for (int e = 0; e < d[0]; ++e) vl.push_back(d[3 + e]);
    }
    std::sort(vl.begin(), vl.end());
    vl.erase(std::unique(vl.begin(), vl.end()), vl.end());
    R[s] = N + (int)vl.size();
    RP[s] = round_up(R[s], 16);
    // limits: the staging registers, and one consumer lane per particle
    if (4L * KS * RP[s] > 1024L * afq::kMdRowsPF || (int)vl.size() > 64) return AFQMC_OK;
    rowmap[s].resize(R[s]);
    for (int a = 0; a < N; ++a) rowmap[s][a] = a;
    for (size_t t = 0; t < vl.size(); ++t) rowmap[s][N + t] = vl[t];
    // the distinct (particle, hole) pairs, ordered by particle then hole, and
    // each particle's first pair
    auto dets = [&](int k, int* t, int* r) {
      const int* d = &exc[((size_t)order[k] * 2 + s) * 5];
      for (int e = 0; e < d[0]; ++e) {
        r[e] = d[1 + e];
        t[e] = (int)(std::lower_bound(vl.begin(), vl.end(), d[3 + e]) - vl.begin());
      }
      return d[0];
    };
    std::map<int, int> pid;
    for (int k = 0; k < n_det; ++k) {
      int t[2] = {0, 0}, r[2] = {0, 0};
      const int E = dets(k, t, r);
      for (int e = 0; e < E; ++e)
        for (int f = 0; f < E; ++f) pid.emplace((t[e] << 8) | r[f], 0);
    }
    if (pid.size() > 0xffff) return AFQMC_OK;
    pbeg[s].assign(vl.size() + 1, 0);
    for (auto& kv : pid) {
      kv.second = (int)pairs[s].size();
      pairs[s].push_back(kv.first);
      ++pbeg[s][(kv.first >> 8) + 1];
    }
    for (size_t t = 0; t < vl.size(); ++t) pbeg[s][t + 1] += pbeg[s][t];
    for (int k = 0; k < n_det; ++k) {
      int t[2] = {0, 0}, r[2] = {0, 0}, pi[2][2] = {{0, 0}, {0, 0}};
      const int E = dets(k, t, r);
      for (int e = 0; e < E; ++e)
        for (int f = 0; f < E; ++f) pi[e][f] = pid.at((t[e] << 8) | r[f]);
      int* w = &dx[(size_t)k * afq::kMdDx + s * 3];
      w[0] = (int)((unsigned)E | (unsigned)r[0] << 2 | (unsigned)r[1] << 7 | (unsigned)t[0] << 12 |
                   (unsigned)t[1] << 20);
      w[1] = (int)((unsigned)pi[0][0] | (unsigned)pi[0][1] << 16);
      w[2] = (int)((unsigned)pi[1][0] | (unsigned)pi[1][1] << 16);
    }
  }
  void* p;
  if (tr->arena.alloc(&p, dx.size() * sizeof(int))) return AFQMC_ERR_OOM;
  tr->d_mddx = (int*)p;
  if (hipMemcpy(tr->d_mddx, dx.data(), dx.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
    return AFQMC_ERR_DEVICE;
  for (int s = 0; s < 2; ++s) {
    tr->mdR[s] = R[s];
    tr->mdRP[s] = RP[s];
    tr->mdnp[s] = (int)pairs[s].size();
    if (!R[s]) {  // no electrons of this spin: a zero table the staging loads may touch
      void* pz;
      if (tr->arena.alloc(&pz, 64)) return AFQMC_ERR_OOM;
      if (hipMemsetAsync(pz, 0, 64, st) != hipSuccess) return AFQMC_ERR_DEVICE;
      tr->LCc[s] = (float*)pz;
      continue;
    }
    void *pl, *pm, *pr, *pq;
    if (tr->arena.alloc(&pl, (size_t)(G + 2) * 4 * KS * RP[s] * 4) ||
        tr->arena.alloc(&pm, rowmap[s].size() * sizeof(int)) ||
        tr->arena.alloc(&pr, std::max<size_t>(pairs[s].size(), 1) * sizeof(int)) ||
        tr->arena.alloc(&pq, pbeg[s].size() * sizeof(int)))
      return AFQMC_ERR_OOM;
    tr->LCc[s] = (float*)pl;
    tr->d_mdpair[s] = (int*)pr;
    tr->d_mdpbeg[s] = (int*)pq;
    if (hipMemcpy(pm, rowmap[s].data(), rowmap[s].size() * sizeof(int), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(pq, pbeg[s].data(), pbeg[s].size() * sizeof(int), hipMemcpyHostToDevice) !=
            hipSuccess ||
        (!pairs[s].empty() && hipMemcpy(pr, pairs[s].data(), pairs[s].size() * sizeof(int),
                                        hipMemcpyHostToDevice) != hipSuccess))
      return AFQMC_ERR_DEVICE;
    if (afq::md_rows_gather(st, G + 1, M, KS, R[s], RP[s], (const int*)pm, tr->LC64[s],
                            tr->LCc[s]) != hipSuccess ||
        afq::md_rows_gather(st, 1, M, KS, R[s], RP[s], (const int*)pm, tr->C[s],
                            tr->LCc[s] + (size_t)(G + 1) * 4 * KS * RP[s]) != hipSuccess)
      return AFQMC_ERR_DEVICE;
  }
  tr->mdKS = KS;
  tr->md_rows = true;
  return AFQMC_OK;
}

}  // namespace

afqmc_status afqmc_footprint_bytes(int M, int n_chol, int n_up, int n_dn, int n_det, int n_walkers,
                                   size_t* bytes) {
  if (!bytes || M < 1 || n_chol < 0 || n_up < 0 || n_dn < 0 || n_up + n_dn < 1 || n_det < 1 ||
      n_walkers < 1)
    return fail(AFQMC_ERR_ARG, "invalid sizes");
  const size_t m = M, g = n_chol, mm = m * m, a = 256;
  auto rnd = [&](size_t b) { return (std::max(b, a) + a - 1) / a * a; };
  const int nel[2] = {n_up, n_dn};
  const size_t MP4 = round_up(M, 4), MP32 = round_up(M, 32), Nt = (size_t)n_up + n_dn;
  size_t tot = rnd(mm * 8) * 2 + rnd(g * mm * 8) + rnd(g * mm * 4) + 2 * rnd(g * mm * 2) +
               rnd(g * (mm + m) / 2 * 12);  // ham (with the packed L copies)
  const size_t NPX = round_up(std::max({n_up, n_dn, 1}), 16);  // the bf16 copies' row tiles
  for (int s = 0; s < 2; ++s) {                                                        // trial
    const size_t NP = round_up(std::max(nel[s], 1), 16);
    const size_t nlt = (g * MP4 + 16) * NP;
    tot += rnd(mm * 8) + rnd(std::max(nel[s], 1) * m * 8) + rnd(nlt * 8) + rnd(nlt * 4) +
           2 * rnd(g * NPX * MP32 * 2);
    if (NP <= 32 && g > 0) {
      const size_t npk = pack_exchange_elems(g, MP4, NP);
      tot += rnd(npk * 8) + rnd(npk * 4);
    } else if (NP <= 64 && g > 0) {
      tot += rnd(pack_exchange_elems(g, MP4, NP) * 4);
    }
    if (n_det > 1) tot += rnd((g + 1) * mm * 8) + rnd((g + 1) * mm * 4);
  }
  tot += 3 * rnd(std::max<size_t>(g, 1) * 8) + rnd(m * Nt * 8) + rnd(mm * 8) + 2 * rnd(mm * 12);
  if (n_det > 1) tot += rnd((size_t)n_det * 40) + rnd((size_t)n_det * 8);
  tot += md_rows_bound_bytes(M, n_chol, n_up, n_dn, n_det);
  const size_t kq[2] = {(size_t)qpad((long)M * n_up), (size_t)qpad((long)M * n_dn)};
  const size_t qb = q_fp32_ok(M, n_up, n_dn) ? 12 : 8;  // FP64 (+ FP32) copies
  if (n_det == 1 && g > 0) tot += rnd((kq[0] + kq[1]) * qpad(g) * qb);  // Lq
  if (use_qroute(M, n_chol, n_up, n_dn, n_det)) {
    int ns[2];
    q_plan(M, n_chol, n_up, n_dn, nullptr, ns);
    tot += rnd((size_t)(ns[0] + ns[1]) * 16);
    size_t tr_max = 0;  // the set-up transient P = R^T R, one spin at a time
    for (int s = 0; s < 2; ++s) {
      if (nel[s]) tot += rnd(kq[s] * kq[s] * 8) + (qb == 12 ? rnd(kq[s] * kq[s] * 4) : 0);
      const size_t kp = MP4 * (size_t)round_up(std::max(nel[s], 1), 16);
      if (nel[s]) tr_max = std::max(tr_max, rnd(kp * kp * 8));
    }
    tot += tr_max;
  }
  tot += 2 * rnd((size_t)n_walkers * m * Nt * 8) + 5 * rnd((size_t)n_walkers * 8);  // walkers
  tot += layout_dims(M, n_chol, (long)Nt, n_det, n_walkers, nullptr).total;
  *bytes = tot;
  return AFQMC_OK;
}

afqmc_status afqmc_walker_workspace_bytes(const afqmc_trial* tr, int n_walkers, size_t* bytes) {
  if (!tr || !bytes) return fail(AFQMC_ERR_ARG, "NULL argument");
  if (n_walkers < 1) return fail(AFQMC_ERR_ARG, "n_walkers must be >= 1");
  *bytes = layout(tr, n_walkers, nullptr).total;
  return AFQMC_OK;
}

afqmc_status afqmc_init_trial(afqmc_trial** out, afqmc_ham* hm, int n_up, int n_dn,
                              const double* C_up, const double* C_dn, int n_det,
                              const double* coeff, const int32_t* exc, int mf_subtract) {
  if (!out) return fail(AFQMC_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!hm) return fail(AFQMC_ERR_ARG, "ham is NULL");
  const int M = hm->M, G = hm->G;
  if (n_up < 0 || n_dn < 0 || n_up + n_dn < 1) return fail(AFQMC_ERR_ARG, "electron counts");
  if (n_up > M || n_dn > M || n_up > AFQMC_MAX_NEL || n_dn > AFQMC_MAX_NEL)
    return fail(AFQMC_ERR_UNSUPPORTED, "too many electrons per spin");
  if (!C_up || !C_dn) return fail(AFQMC_ERR_ARG, "C_up or C_dn is NULL");
  if (n_det < 1) return fail(AFQMC_ERR_ARG, "n_det must be >= 1");
  if (n_det > 1 && (!coeff || !exc)) return fail(AFQMC_ERR_ARG, "coeff / exc NULL with n_det > 1");
  if (!all_finite(C_up, (size_t)M * M) || !all_finite(C_dn, (size_t)M * M))
    return fail(AFQMC_ERR_ARG, "C has a non-finite entry");
  std::vector<int> exc_dev;
  if (n_det > 1) {
    const int row = 1 + 2 * AFQMC_MAX_EXC;
    const int nel_[2] = {n_up, n_dn};
    exc_dev.assign((size_t)n_det * 10, 0);
    for (int i = 0; i < n_det; ++i) {
      if (!std::isfinite(coeff[i])) return fail(AFQMC_ERR_ARG, "coeff has a non-finite entry");
      for (int s = 0; s < 2; ++s) {
        const int32_t* ex = exc + ((size_t)i * 2 + s) * row;
        const int E = ex[0];
        if (E < 0 || E > AFQMC_MAX_EXC) return fail(AFQMC_ERR_ARG, "excitation count out of range");
        if (i == 0 && E != 0) return fail(AFQMC_ERR_ARG, "determinant 0 must be the reference");
        if (E > 2) return fail(AFQMC_ERR_UNSUPPORTED, "more than 2 excitations per spin");
        for (int e = 0; e < E; ++e) {
          const int r = ex[1 + e], v = ex[1 + AFQMC_MAX_EXC + e];
          if (r < 0 || r >= nel_[s] || v < nel_[s] || v >= M)
            return fail(AFQMC_ERR_ARG, "hole / particle index out of range");
          for (int f = 0; f < e; ++f)
            if (ex[1 + f] == r || ex[1 + AFQMC_MAX_EXC + f] == v)
              return fail(AFQMC_ERR_ARG, "repeated hole or particle");
        }
        int* d = &exc_dev[((size_t)i * 2 + s) * 5];
        d[0] = E;
        for (int e = 0; e < E; ++e) {
          d[1 + e] = ex[1 + e];
          d[3 + e] = ex[1 + AFQMC_MAX_EXC + e];
        }
      }
    }
  }
  const int nel[2] = {n_up, n_dn};
  const double* Cs[2] = {C_up, C_dn};
  // the reference determinant must have orthonormal orbitals
  for (int s = 0; s < 2; ++s)
    for (int a = 0; a < nel[s]; ++a)
      for (int b = 0; b < nel[s]; ++b) {
        double d = 0.0;
        for (int m = 0; m < M; ++m) d += Cs[s][(size_t)m * M + a] * Cs[s][(size_t)m * M + b];
        if (std::fabs(d - (a == b ? 1.0 : 0.0)) > 1e-8)
          return fail(AFQMC_ERR_SINGULAR, "occupied trial orbitals are not orthonormal");
      }
  AFQ_CK(hipSetDevice(hm->device));
  hipStream_t st = nullptr;
  afqmc_trial* tr = new afqmc_trial();
  tr->ham = hm;
  tr->nel[0] = n_up;
  tr->nel[1] = n_dn;
  tr->Nt = n_up + n_dn;
  tr->MP4 = round_up(M, 4);
  tr->MP32 = round_up(M, 32);
  tr->n_det = n_det;
  for (int s = 0; s < 2; ++s) tr->NP[s] = round_up(std::max(nel[s], 1), 16);
  auto bad = [&](afqmc_status code, const char* what) {
    tr->arena.release();
    delete tr;
    return fail(code, what);
  };
  const size_t mm = (size_t)M * M;
  for (int s = 0; s < 2; ++s) {
    void *pc, *ph, *p64, *p32;
    // 16 zero rows after the last slab: the exchange kernel reads its A
    // operand in batches of four k steps without bounds checks
    const size_t nlt = (size_t)G * tr->MP4 * tr->NP[s] + (size_t)16 * tr->NP[s];
    if (tr->arena.alloc(&pc, mm * 8) || tr->arena.alloc(&ph, (size_t)std::max(nel[s], 1) * M * 8) ||
        tr->arena.alloc(&p64, nlt * 8) || tr->arena.alloc(&p32, nlt * 4))
      return bad(AFQMC_ERR_OOM, "trial allocation failed");
    tr->C[s] = (double*)pc;
    tr->htil[s] = (double*)ph;
    tr->Lt64[s] = (double*)p64;
    tr->Lt32[s] = (float*)p32;
    if (hipMemcpy(tr->C[s], Cs[s], mm * 8, hipMemcpyHostToDevice) != hipSuccess)
      return bad(AFQMC_ERR_DEVICE, "C upload");
    if (hipMemsetAsync(tr->Lt64[s], 0, nlt * 8, st) != hipSuccess) return bad(AFQMC_ERR_DEVICE, "memset");
    if (nel[s] > 0 && G > 0) {
      // Lt[g][m][a] = (L_g C)[m][a] = (C^T L_g)[a][m]
      if (afq::gemm_real<double, double, false>(st, M, nel[s], M, hm->L, M, (long)mm, tr->C[s], M,
                                                0, tr->Lt64[s], tr->NP[s],
                                                (long)tr->MP4 * tr->NP[s], G, 1.0) != hipSuccess)
        return bad(AFQMC_ERR_DEVICE, "half-rotation");
    }
    if (afq::convert_f64_f32(st, tr->Lt64[s], tr->Lt32[s], (long)nlt) != hipSuccess)
      return bad(AFQMC_ERR_DEVICE, "convert");
    if (tr->NP[s] <= 32 && G > 0) {
      const size_t npk = pack_exchange_elems(G, tr->MP4, tr->NP[s]);
      void *q64, *q32;
      if (tr->arena.alloc(&q64, npk * 8) || tr->arena.alloc(&q32, npk * 4))
        return bad(AFQMC_ERR_OOM, "trial allocation failed");
      tr->Apk64[s] = (double*)q64;
      tr->Apk32[s] = (float*)q32;
      if (afq::pack_exchange_a<double>(st, G, tr->MP4, tr->NP[s], tr->Lt64[s], tr->Apk64[s]) !=
              hipSuccess ||
          afq::pack_exchange_a<float>(st, G, tr->MP4, tr->NP[s], tr->Lt32[s], tr->Apk32[s]) !=
              hipSuccess)
        return bad(AFQMC_ERR_DEVICE, "exchange operand repack");
    } else if (tr->NP[s] <= 64 && G > 0) {
      // FP32 only: the wide exchange kernel's layout (one row tile per wavefront)
      const size_t npk = pack_exchange_elems(G, tr->MP4, tr->NP[s]);
      void* q32;
      if (tr->arena.alloc(&q32, npk * 4)) return bad(AFQMC_ERR_OOM, "trial allocation failed");
      tr->Apk32[s] = (float*)q32;
      if (afq::pack_exchange_a<float>(st, G, tr->MP4, tr->NP[s], tr->Lt32[s], tr->Apk32[s]) !=
          hipSuccess)
        return bad(AFQMC_ERR_DEVICE, "exchange operand repack");
    }
    {
      // both spins with the larger spin's row tiles, so one kernel instance serves both
      const int NPX = std::max(tr->NP[0], tr->NP[1]);
      void *pb = nullptr, *pbl = nullptr;
      const size_t nb = (size_t)G * NPX * tr->MP32;
      if (tr->arena.alloc(&pb, nb * 2) || tr->arena.alloc(&pbl, nb * 2))
        return bad(AFQMC_ERR_OOM, "trial allocation failed");
      tr->Ltbf[s] = pb;
      tr->Ltbf_lo[s] = pbl;
      if (afq::pack_ltilde_bf16(st, G, tr->MP4, tr->NP[s], NPX, tr->MP32, tr->Lt64[s], pb, pbl) !=
          hipSuccess)
        return bad(AFQMC_ERR_DEVICE, "bf16 half-rotation");
    }
    if (nel[s] > 0) {
      // htil[a][m] = sum_i C[i][a] h[i][m]
      if (afq::gemm_real<double, double, true>(st, nel[s], M, M, tr->C[s], M, 0, hm->h, M, 0,
                                               tr->htil[s], M, 0, 1, 1.0) != hipSuccess)
        return bad(AFQMC_ERR_DEVICE, "htil");
    }
  }
  void *plb, *pd0, *pvr, *pvi, *plL;
  if (tr->arena.alloc(&plb, (size_t)std::max(G, 1) * 8) || tr->arena.alloc(&pd0, (size_t)M * tr->Nt * 8) ||
      tr->arena.alloc(&pvr, (size_t)std::max(G, 1) * 8) || tr->arena.alloc(&pvi, (size_t)std::max(G, 1) * 8) ||
      tr->arena.alloc(&plL, mm * 8))
    return bad(AFQMC_ERR_OOM, "trial allocation failed");
  tr->lbar = (double*)plb;
  tr->D0 = (double*)pd0;
  tr->vref_re = (double*)pvr;
  tr->vref_im = (double*)pvi;
  if (hipMemsetAsync(tr->lbar, 0, (size_t)std::max(G, 1) * 8, st) != hipSuccess)
    return bad(AFQMC_ERR_DEVICE, "memset");
  if (mf_subtract) {
    for (int s = 0; s < 2; ++s)
      if (afq::lbar_accumulate(st, G, M, tr->MP4, nel[s], tr->NP[s], tr->Lt64[s], tr->C[s],
                               tr->lbar) != hipSuccess)
        return bad(AFQMC_ERR_DEVICE, "lbar");
  }
  // sum_g lbar_g L_g
  if (hipMemsetAsync(plL, 0, mm * 8, st) != hipSuccess) return bad(AFQMC_ERR_DEVICE, "memset");
  if (G > 0 && afq::gemm_real<double, double, true>(st, 1, (int)mm, G, tr->lbar, 1, 0, hm->L,
                                                    (int)mm, 0, (double*)plL, (int)mm, 0, 1,
                                                    1.0) != hipSuccess)
    return bad(AFQMC_ERR_DEVICE, "lbar L");
  std::vector<double> L2h(mm), lLh(mm);
  if (hipStreamSynchronize(st) != hipSuccess ||
      hipMemcpy(L2h.data(), hm->L2, mm * 8, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(lLh.data(), plL, mm * 8, hipMemcpyDeviceToHost) != hipSuccess)
    return bad(AFQMC_ERR_DEVICE, "download");
  tr->H1p.resize(mm);
  for (size_t i = 0; i < mm; ++i) tr->H1p[i] = hm->h_host[i] - 0.5 * L2h[i] + lLh[i];
  // symmetrise (rounding of the two GEMMs)
  for (int i = 0; i < M; ++i)
    for (int j = i + 1; j < M; ++j) {
      const double a = 0.5 * (tr->H1p[(size_t)i * M + j] + tr->H1p[(size_t)j * M + i]);
      tr->H1p[(size_t)i * M + j] = tr->H1p[(size_t)j * M + i] = a;
    }
  std::vector<double> D0h((size_t)M * tr->Nt);
  for (int m = 0; m < M; ++m) {
    for (int a = 0; a < n_up; ++a) D0h[(size_t)m * tr->Nt + a] = C_up[(size_t)m * M + a];
    for (int a = 0; a < n_dn; ++a) D0h[(size_t)m * tr->Nt + n_up + a] = C_dn[(size_t)m * M + a];
  }
  if (hipMemcpy(tr->D0, D0h.data(), D0h.size() * 8, hipMemcpyHostToDevice) != hipSuccess)
    return bad(AFQMC_ERR_DEVICE, "D0 upload");
  {
    std::vector<double> lb((size_t)std::max(G, 1));
    if (hipMemcpy(lb.data(), tr->lbar, lb.size() * 8, hipMemcpyDeviceToHost) != hipSuccess)
      return bad(AFQMC_ERR_DEVICE, "lbar download");
    double s2 = 0.0;
    for (int g = 0; g < G; ++g) s2 += lb[g] * lb[g];
    tr->e0_shift = hm->e_core - 0.5 * s2;
  }
  for (int s = 0; s < 2; ++s) tr->Kp[s] = qpad((long)M * nel[s]);
  tr->Gp = qpad(G);
  tr->q32 = q_fp32_ok(M, n_up, n_dn);
  if (n_det == 1 && G > 0) {
    const size_t nk = (size_t)(tr->Kp[0] + tr->Kp[1]) * tr->Gp;
    void* q64;
    if (tr->arena.alloc(&q64, nk * 8)) return bad(AFQMC_ERR_OOM, "trial allocation failed");
    tr->Lq64 = (double*)q64;
    if (afq::build_lsplit(st, G, tr->Gp, M, tr->MP4, n_up, n_dn, tr->NP[0], tr->NP[1], tr->Kp[0],
                          tr->Kp[1], tr->Lt64[0], tr->Lt64[1], tr->Lq64) != hipSuccess)
      return bad(AFQMC_ERR_DEVICE, "force-bias operand");
    if (tr->q32) {
      void* q32;
      if (tr->arena.alloc(&q32, nk * 4)) return bad(AFQMC_ERR_OOM, "trial allocation failed");
      tr->Lq32 = (float*)q32;
      if (afq::convert_f64_f32(st, tr->Lq64, tr->Lq32, (long)nk) != hipSuccess)
        return bad(AFQMC_ERR_DEVICE, "force-bias operand");
    }
  }
  if (use_qroute(M, G, n_up, n_dn, n_det)) {
    std::vector<int4> segs;
    q_plan(M, G, n_up, n_dn, &segs, tr->nseg);
    void* ps;
    if (tr->arena.alloc(&ps, segs.size() * sizeof(int4)))
      return bad(AFQMC_ERR_OOM, "trial allocation failed");
    tr->qsegs = (int4*)ps;
    if (hipMemcpy(tr->qsegs, segs.data(), segs.size() * sizeof(int4), hipMemcpyHostToDevice) !=
        hipSuccess)
      return bad(AFQMC_ERR_DEVICE, "segment upload");
    for (int s = 0; s < 2; ++s) {
      if (nel[s] == 0) continue;
      const long Kq = tr->Kp[s], Kp = (long)tr->MP4 * tr->NP[s];
      void *q64, *q32 = nullptr;
      if (tr->arena.alloc(&q64, (size_t)Kq * Kq * 8) ||
          (tr->q32 && tr->arena.alloc(&q32, (size_t)Kq * Kq * 4)))
        return bad(AFQMC_ERR_OOM, "trial allocation failed");
      tr->Q64[s] = (double*)q64;
      tr->Q32[s] = (float*)q32;
      // P = R^T R over the padded index (m NP + a), then the index permutation;
      // P is a stream-ordered transient (no device-wide synchronisation when it
      // is freed; afqmc_footprint_bytes counts it)
      double* P = nullptr;
      if (hipMallocAsync((void**)&P, (size_t)Kp * Kp * 8, st) != hipSuccess)
        return bad(AFQMC_ERR_OOM, "Q set-up allocation failed");
      const bool ok =
          afq::gemm_real<double, double, true>(st, (int)Kp, (int)Kp, G, tr->Lt64[s], (int)Kp, 0,
                                               tr->Lt64[s], (int)Kp, 0, P, (int)Kp, 0, 1, 1.0) ==
              hipSuccess &&
          afq::perm_qpad<double>(st, M, nel[s], tr->NP[s], tr->MP4, (int)Kq, P, tr->Q64[s]) ==
              hipSuccess &&
          (!tr->q32 || afq::perm_qpad<float>(st, M, nel[s], tr->NP[s], tr->MP4, (int)Kq, P,
                                             tr->Q32[s]) == hipSuccess) &&
          hipStreamSynchronize(st) == hipSuccess;
      const bool freed = hipFreeAsync(P, st) == hipSuccess && hipStreamSynchronize(st) == hipSuccess;
      if (!ok || !freed) return bad(AFQMC_ERR_DEVICE, "Q set-up");
    }
    tr->qbuilt = true;
    tr->qroute = true;
  }
  if (n_det > 1) {
    void *pe, *pc;
    if (tr->arena.alloc(&pe, exc_dev.size() * sizeof(int)) || tr->arena.alloc(&pc, (size_t)n_det * 8))
      return bad(AFQMC_ERR_OOM, "trial allocation failed");
    tr->d_exc = (int*)pe;
    tr->d_coeff = (double*)pc;
    tr->coeff.assign(coeff, coeff + n_det);
    if (hipMemcpy(tr->d_exc, exc_dev.data(), exc_dev.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(tr->d_coeff, coeff, (size_t)n_det * 8, hipMemcpyHostToDevice) != hipSuccess)
      return bad(AFQMC_ERR_DEVICE, "excitation upload");
    const size_t nlc = (size_t)(G + 1) * mm;
    for (int s = 0; s < 2; ++s) {
      void *p64, *p32;
      if (tr->arena.alloc(&p64, nlc * 8) || tr->arena.alloc(&p32, nlc * 4))
        return bad(AFQMC_ERR_OOM, "trial allocation failed");
      tr->LC64[s] = (double*)p64;
      tr->LC32[s] = (float*)p32;
      // LC[g][m][p] = (L_g C)[m][p] for g < G, LC[G] = h C
      if (G > 0 && afq::gemm_real<double, double, false>(st, M, M, M, hm->L, M, (long)mm, tr->C[s], M,
                                                         0, tr->LC64[s], M, (long)mm, G, 1.0) != hipSuccess)
        return bad(AFQMC_ERR_DEVICE, "L C");
      if (afq::gemm_real<double, double, false>(st, M, M, M, hm->h, M, 0, tr->C[s], M, 0,
                                                tr->LC64[s] + (size_t)G * mm, M, 0, 1, 1.0) != hipSuccess)
        return bad(AFQMC_ERR_DEVICE, "h C");
      if (afq::convert_f64_f32(st, tr->LC64[s], tr->LC32[s], (long)nlc) != hipSuccess)
        return bad(AFQMC_ERR_DEVICE, "convert");
    }
    const afqmc_status rs = md_rows_setup(tr, exc_dev, st);
    if (rs != AFQMC_OK) return bad(rs, "compact-row tables");
    if (hipStreamSynchronize(st) != hipSuccess) return bad(AFQMC_ERR_DEVICE, "sync");
  }
  // reference state: one walker at D_0, measured in FP64
  {
    afqmc_walkers rw;
    std::memset(&rw, 0, sizeof(rw));
    rw.n_walkers = 1;
    const WS ws0 = layout(tr, 1, nullptr);
    void *pr, *pi, *pw, *pl, *pe, *pwork;
    Arena tmp;
    if (tmp.alloc(&pr, D0h.size() * 8) || tmp.alloc(&pi, D0h.size() * 8) || tmp.alloc(&pw, 8) ||
        tmp.alloc(&pl, 16) || tmp.alloc(&pe, 16) || tmp.alloc(&pwork, ws0.total)) {
      tmp.release();
      return bad(AFQMC_ERR_OOM, "reference walker");
    }
    rw.phi_re = (double*)pr;
    rw.phi_im = (double*)pi;
    rw.weight = (double*)pw;
    rw.logovlp_re = (double*)pl;
    rw.logovlp_im = (double*)pl + 1;
    rw.eloc_re = (double*)pe;
    rw.eloc_im = (double*)pe + 1;
    rw.workspace = pwork;
    rw.workspace_bytes = ws0.total;
    const WS ws = layout(tr, 1, pwork);
    bool ok = hipMemcpy(pr, tr->D0, D0h.size() * 8, hipMemcpyDeviceToDevice) == hipSuccess &&
              hipMemset(pi, 0, D0h.size() * 8) == hipSuccess &&
              afq::fill(st, (double*)pw, 1, 1.0) == hipSuccess;
    afqmc_status ms = ok ? measure_set(tr, &rw, ws, AFQMC_FP64, st) : AFQMC_ERR_DEVICE;
    double hv[4];
    ok = ok && ms == AFQMC_OK && hipStreamSynchronize(st) == hipSuccess &&
         hipMemcpy(&hv[0], pl, 16, hipMemcpyDeviceToHost) == hipSuccess &&
         hipMemcpy(&hv[2], pe, 16, hipMemcpyDeviceToHost) == hipSuccess &&
         hipMemcpy(tr->vref_re, ws.v_re, (size_t)std::max(G, 1) * 8, hipMemcpyDeviceToDevice) == hipSuccess &&
         hipMemcpy(tr->vref_im, ws.v_im, (size_t)std::max(G, 1) * 8, hipMemcpyDeviceToDevice) == hipSuccess &&
         hipDeviceSynchronize() == hipSuccess;
    tmp.release();
    if (!ok) return bad(AFQMC_ERR_DEVICE, "reference walker measure failed");
    tr->ref_ls[0] = hv[0];
    tr->ref_ls[1] = hv[1];
    tr->ref_el[0] = hv[2];
    tr->ref_el[1] = hv[3];
  }
  *out = tr;
  return AFQMC_OK;
}

void afqmc_free_trial(afqmc_trial* tr) {
  if (!tr) return;
  (void)hipSetDevice(tr->ham->device);
  tr->arena.release();
  delete tr;
}

afqmc_status afqmc_walkers_from_trial(afqmc_ham* hm, afqmc_trial* tr, afqmc_walkers* wk,
                                      void* stream) {
  if (!hm || !tr) return fail(AFQMC_ERR_ARG, "NULL ham / trial");
  if (tr->ham != hm) return fail(AFQMC_ERR_STATE, "trial was built on another Hamiltonian");
  afqmc_status s = check_walkers(tr, wk);
  if (s != AFQMC_OK) return s;
  AFQ_CK(hipSetDevice(hm->device));
  hipStream_t st = (hipStream_t)stream;
  const int W = wk->n_walkers, G = hm->G;
  const long row = (long)hm->M * tr->Nt;
  const WS ws = layout(tr, W, wk->workspace);
  AFQ_CK(afq::broadcast_rows(st, W, row, tr->D0, wk->phi_re));
  AFQ_CK(afq::fill(st, wk->phi_im, (long)W * row, 0.0));
  AFQ_CK(afq::fill(st, wk->weight, W, 1.0));
  AFQ_CK(afq::fill(st, wk->logovlp_re, W, tr->ref_ls[0]));
  AFQ_CK(afq::fill(st, wk->logovlp_im, W, tr->ref_ls[1]));
  AFQ_CK(afq::fill(st, wk->eloc_re, W, tr->ref_el[0]));
  AFQ_CK(afq::fill(st, wk->eloc_im, W, tr->ref_el[1]));
  if (G > 0) {
    AFQ_CK(afq::broadcast_rows(st, W, G, tr->vref_re, ws.v_re));
    AFQ_CK(afq::broadcast_rows(st, W, G, tr->vref_im, ws.v_im));
  }
  return AFQMC_OK;
}

afqmc_status afqmc_local_energy(afqmc_ham* hm, afqmc_trial* tr, afqmc_walkers* wk,
                                double* emix_host, void* stream) {
  if (!hm || !tr) return fail(AFQMC_ERR_ARG, "NULL ham / trial");
  if (tr->ham != hm) return fail(AFQMC_ERR_STATE, "trial was built on another Hamiltonian");
  afqmc_status s = check_walkers(tr, wk);
  if (s != AFQMC_OK) return s;
  AFQ_CK(hipSetDevice(hm->device));
  hipStream_t st = (hipStream_t)stream;
  const WS ws = layout(tr, wk->n_walkers, wk->workspace);
  s = measure_set(tr, wk, ws, AFQMC_FP64, st);
  if (s != AFQMC_OK) return s;
  if (emix_host) {
    AFQ_CK(afq::mixed_energy(st, wk->n_walkers, wk->weight, wk->eloc_re, ws.scal, ws.scal + 1));
    double hv[2];
    AFQ_CK(hipMemcpyAsync(hv, ws.scal, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    AFQ_CK(hipStreamSynchronize(st));
    if (!(hv[1] > 0.0)) return fail(AFQMC_ERR_NONFINITE, "sum of weights is zero");
    *emix_host = hv[0];
  }
  return AFQMC_OK;
}

afqmc_status afqmc_orthonormalize(afqmc_ham* hm, afqmc_trial* tr, afqmc_walkers* wk, void* stream) {
  if (!hm || !tr) return fail(AFQMC_ERR_ARG, "NULL ham / trial");
  if (tr->ham != hm) return fail(AFQMC_ERR_STATE, "trial was built on another Hamiltonian");
  afqmc_status s = check_walkers(tr, wk);
  if (s != AFQMC_OK) return s;
  AFQ_CK(hipSetDevice(hm->device));
  const WS ws = layout(tr, wk->n_walkers, wk->workspace);
  return orthonormalize_impl(tr, wk, ws, (hipStream_t)stream);
}

afqmc_status afqmc_reconfigure(afqmc_trial* tr, afqmc_walkers* wk, uint64_t seed, uint64_t pc_index,
                               double* norm_factor_host, void* stream) {
  if (!tr) return fail(AFQMC_ERR_ARG, "NULL trial");
  afqmc_status s = check_walkers(tr, wk);
  if (s != AFQMC_OK) return s;
  AFQ_CK(hipSetDevice(tr->ham->device));
  hipStream_t st = (hipStream_t)stream;
  const WS ws = layout(tr, wk->n_walkers, wk->workspace);
  s = reconfigure_impl(tr, wk, ws, seed, pc_index, st);
  if (s != AFQMC_OK) return s;
  if (norm_factor_host) {
    AFQ_CK(hipMemcpyAsync(norm_factor_host, ws.scal + 2, sizeof(double), hipMemcpyDeviceToHost, st));
    AFQ_CK(hipStreamSynchronize(st));
    if (!(*norm_factor_host > 0.0))
      return fail(AFQMC_ERR_NONFINITE, "comb: the sum of weights is not positive and finite");
  }
  return AFQMC_OK;
}

afqmc_status afqmc_propagate(afqmc_ham* hm, afqmc_trial* tr, afqmc_walkers* wk, int n_steps,
                             double dt, uint64_t seed, uint64_t step0, const afqmc_options* opt,
                             double* emix_dev, void* stream) {
  if (!hm || !tr || !opt) return fail(AFQMC_ERR_ARG, "NULL ham / trial / options");
  if (tr->ham != hm) return fail(AFQMC_ERR_STATE, "trial was built on another Hamiltonian");
  afqmc_status s = check_walkers(tr, wk);
  if (s != AFQMC_OK) return s;
  if (n_steps < 0) return fail(AFQMC_ERR_ARG, "n_steps must be >= 0");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(AFQMC_ERR_ARG, "dt must be positive");
  if (opt->taylor_order < 1 || opt->taylor_order > 64) return fail(AFQMC_ERR_ARG, "taylor_order");
  if (opt->ortho_every < 0 || opt->pc_every < 0) return fail(AFQMC_ERR_ARG, "negative interval");
  if (!std::isfinite(opt->e_trial)) return fail(AFQMC_ERR_ARG, "e_trial is not finite");
  if (opt->weight_mode != AFQMC_WEIGHT_LOCAL_ENERGY && opt->weight_mode != AFQMC_WEIGHT_HYBRID)
    return fail(AFQMC_ERR_ARG, "weight_mode must be AFQMC_WEIGHT_LOCAL_ENERGY or AFQMC_WEIGHT_HYBRID");
  if (opt->weight_mode == AFQMC_WEIGHT_HYBRID && opt->meas_every < 1)
    return fail(AFQMC_ERR_ARG, "meas_every must be >= 1 in the hybrid form");
  const bool bfp = opt->chol_prec == AFQMC_BF16 || opt->chol_prec == AFQMC_BF16X3;
  if ((opt->chol_prec != AFQMC_FP64 && opt->chol_prec != AFQMC_FP32 && !bfp) ||
      (opt->taylor_prec != AFQMC_FP64 && opt->taylor_prec != AFQMC_FP32))
    return fail(AFQMC_ERR_UNSUPPORTED, "precision");
  if (bfp && tr->n_det > 1)
    return fail(AFQMC_ERR_UNSUPPORTED, "bf16 contractions with a multi-determinant trial");
  AFQ_CK(hipSetDevice(hm->device));
  hipStream_t st = (hipStream_t)stream;
  const WS ws = layout(tr, wk->n_walkers, wk->workspace);
  afqmc_status err = AFQMC_OK;
  B1Entry* b1 = get_b1(tr, dt, st, &err);
  if (!b1) return err;
  s = measure_set(tr, wk, ws, opt->chol_prec, st);
  if (s != AFQMC_OK) return s;
  const bool c32 = opt->chol_prec == AFQMC_FP32, t32 = opt->taylor_prec == AFQMC_FP32;
  if (bfp) {
    if (t32)
      return propagate_typed<Bf16Tag, float>(tr, wk, ws, b1, n_steps, dt, seed, step0, opt, emix_dev, st);
    return propagate_typed<Bf16Tag, double>(tr, wk, ws, b1, n_steps, dt, seed, step0, opt, emix_dev, st);
  }
  if (c32 && t32)
    return propagate_typed<float, float>(tr, wk, ws, b1, n_steps, dt, seed, step0, opt, emix_dev, st);
  if (c32 && !t32)
    return propagate_typed<float, double>(tr, wk, ws, b1, n_steps, dt, seed, step0, opt, emix_dev, st);
  if (!c32 && t32)
    return propagate_typed<double, float>(tr, wk, ws, b1, n_steps, dt, seed, step0, opt, emix_dev, st);
  return propagate_typed<double, double>(tr, wk, ws, b1, n_steps, dt, seed, step0, opt, emix_dev, st);
}

afqmc_status afqmc_timing_enable(afqmc_ham* hm, int class_mask) {
  if (!hm) return fail(AFQMC_ERR_ARG, "NULL ham");
  hm->timer.mask = (unsigned)class_mask & ((1u << AFQMC_NUM_KERNEL_CLASSES) - 1u);
  if (hm->timer.mask) hm->timer.reserve(4096);
  return AFQMC_OK;
}

afqmc_status afqmc_trial_exchange_route(const afqmc_trial* tr, int* route) {
  if (!tr || !route) return fail(AFQMC_ERR_ARG, "NULL trial or route");
  *route = tr->qroute ? 1 : 0;
  return AFQMC_OK;
}

afqmc_status afqmc_trial_set_exchange_route(afqmc_trial* tr, int route) {
  if (!tr) return fail(AFQMC_ERR_ARG, "NULL trial");
  if (route != 0 && route != 1) return fail(AFQMC_ERR_ARG, "route must be 0 (Ltil) or 1 (Q)");
  if (route == 1 && !tr->qbuilt)
    return fail(AFQMC_ERR_UNSUPPORTED, "this trial has no Q tensor (see use conditions)");
  tr->qroute = route == 1;
  return AFQMC_OK;
}

afqmc_status afqmc_timing_read(afqmc_ham* hm, int kernel_class, int64_t* launches,
                               double* total_ms) {
  if (!hm || !launches || !total_ms) return fail(AFQMC_ERR_ARG, "NULL argument");
  if (kernel_class < 0 || kernel_class >= AFQMC_NUM_KERNEL_CLASSES)
    return fail(AFQMC_ERR_ARG, "kernel_class out of range");
  AFQ_CK(hipSetDevice(hm->device));
  AFQ_CK(hm->timer.drain());
  *launches = hm->timer.count[kernel_class];
  *total_ms = hm->timer.total_ms[kernel_class];
  hm->timer.count[kernel_class] = 0;
  hm->timer.total_ms[kernel_class] = 0.0;
  return AFQMC_OK;
}

afqmc_status afqmc_fields(uint64_t seed, uint64_t t, int n_walkers, int n_chol, int system_id,
                          double* x_dev, void* stream) {
  if (n_walkers < 1 || n_chol < 1 || system_id < 0 || !x_dev)
    return fail(AFQMC_ERR_ARG, "invalid fields request");
  AFQ_CK(afq::fields_coeff<double>((hipStream_t)stream, n_walkers, n_chol, 0, seed, t, system_id,
                                   1.0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                                   x_dev));
  return AFQMC_OK;
}

}  // extern "C"

// ===========================================================================
// Groups: walkers of several systems propagated together by the
// walker-resident kernel (one workgroup per walker, a segment of steps per
// launch), each segment [steps, mixed energies, combs, step counter]
// captured once as a HIP graph and replayed; launch shape (threads per
// walker block, segment length) from a small autotuner with a JSON cache.
// ===========================================================================
#include <fstream>
#include <map>
#include <mutex>
#include <numeric>
#include <sstream>

#include "resident.hpp"

struct afqmc_group {
  int device = 0;
  int n = 0;
  std::vector<afqmc_group_member> members;
  std::vector<afq::ResMember> h_mem;
  afq::ResMember* d_mem = nullptr;
  uint64_t* tdev = nullptr;
  double* wsum = nullptr;
  int wsum_K = 0;
  int w_total = 0, w_max = 0;
  size_t lds_bytes = 0;
  int threads = 256;
  int K = 20;
  bool k_fixed = false;  // K = gcd of the members' comb intervals
  int tuned = 0;         // 0: default shape, 1: measured, 2: from the cache
  std::string signature;
  hipStream_t cap = nullptr;  // private stream the segment graph is captured on
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // kernel timing of the resident launches (direct launches, no graph, while on)
  KernelTimer timer;
  bool timing = false;
  int64_t timed_steps = 0;
  Arena arena;
};

namespace {

std::mutex g_tune_mu;
std::string g_tune_path;
bool g_tune_path_set = false;

std::string tune_path() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (!g_tune_path_set) {
    const char* e = std::getenv("AFQMC_TUNE_CACHE");
    if (e) g_tune_path = e;
    g_tune_path_set = true;
  }
  return g_tune_path;
}

// The cache file: {"afqmc_tune": 1, "entries": {  one line per entry
//   "<signature>": {"threads": T, "segment": K, "us_per_step": X},  ... }}
struct TuneEntry { int threads = 0, segment = 0; double us = 0.0; };

std::map<std::string, TuneEntry> tune_read(const std::string& path) {
  std::map<std::string, TuneEntry> out;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    const size_t q0 = line.find('"');
    const size_t q1 = q0 == std::string::npos ? q0 : line.find('"', q0 + 1);
    const size_t br = q1 == std::string::npos ? q1 : line.find('{', q1);
    if (br == std::string::npos) continue;
    TuneEntry e;
    if (std::sscanf(line.c_str() + br, "{\"threads\": %d, \"segment\": %d, \"us_per_step\": %lf",
                    &e.threads, &e.segment, &e.us) == 3)
      out[line.substr(q0 + 1, q1 - q0 - 1)] = e;
  }
  return out;
}

void tune_write(const std::string& path, const std::string& sig, const TuneEntry& e) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  std::map<std::string, TuneEntry> all = tune_read(path);
  all[sig] = e;
  const std::string tmp = path + ".tmp";
  {
    std::ofstream f(tmp);
    f << "{\"afqmc_tune\": 1, \"entries\": {\n";
    size_t i = 0;
    for (const auto& kv : all) {
      char buf[160];
      std::snprintf(buf, sizeof buf, "{\"threads\": %d, \"segment\": %d, \"us_per_step\": %.3f}",
                    kv.second.threads, kv.second.segment, kv.second.us);
      f << "\"" << kv.first << "\": " << buf << (++i < all.size() ? ",\n" : "\n");
    }
    f << "}}\n";
  }
  std::rename(tmp.c_str(), path.c_str());
}

// Whether a trial with these options can run in the resident kernel.
afqmc_status resident_check(const afqmc_trial* tr, const afqmc_options* o, size_t* lds) {
  const afqmc_ham* hm = tr->ham;
  const int M = hm->M, Nt = tr->Nt;
  if (tr->n_det != 1) return fail(AFQMC_ERR_UNSUPPORTED, "resident path: single-determinant trials only");
  if (o && o->weight_mode != AFQMC_WEIGHT_LOCAL_ENERGY)
    return fail(AFQMC_ERR_UNSUPPORTED, "resident path: local-energy weights only");
  if (M > afq::kResMaxM || std::max(tr->nel[0], tr->nel[1]) > M)
    return fail(AFQMC_ERR_UNSUPPORTED, "resident path: M <= 64 and N_sigma <= M");
  const afq::ResLds Lo = afq::res_lds(M, Nt, hm->G, std::max(tr->nel[0], tr->nel[1]));
  const size_t bytes = (size_t)Lo.total * sizeof(double);
  if (bytes > hm->max_lds)
    return fail(AFQMC_ERR_UNSUPPORTED, "resident path: the walker does not fit one CU's LDS");
  if (lds) *lds = bytes;
  return AFQMC_OK;
}

void group_drop_graph(afqmc_group* g) {
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  g->exec = nullptr;
  g->graph = nullptr;
}

afqmc_status group_segment(afqmc_group* g, int len, hipStream_t st) {
  {
    TimedLaunch tl(g->timing ? &g->timer : nullptr, 0, st);
    AFQ_CK(afq::res_steps(st, g->d_mem, g->n, g->w_total, g->threads, g->lds_bytes, g->tdev, len,
                          0, g->wsum));
  }
  if (g->timing) g->timed_steps += len;
  AFQ_CK(afq::res_emix(st, g->d_mem, g->n, g->w_total, g->tdev, len, g->wsum));
  AFQ_CK(afq::res_comb(st, g->d_mem, g->n, g->w_total, g->tdev, len, g->w_max));
  AFQ_CK(afq::res_advance(st, g->tdev, len));
  return AFQMC_OK;
}

afqmc_status group_run(afqmc_group* g, int n_steps, uint64_t step0, double* const* emix,
                       hipStream_t st, bool use_graph) {
  std::vector<double*> em(g->n, nullptr);
  for (int m = 0; m < g->n; ++m) em[m] = emix ? emix[m] : nullptr;
  AFQ_CK(afq::res_begin(st, g->d_mem, g->n, g->tdev, step0, em.data()));
  // the call first refreshes log S, E_L and v from phi
  AFQ_CK(afq::res_steps(st, g->d_mem, g->n, g->w_total, g->threads, g->lds_bytes, g->tdev, 0, 1,
                        g->wsum));
  int left = n_steps;
  uint64_t t = step0;
  if (g->k_fixed) {  // segments end where combs fall
    const int head = (int)((g->K - (int)(t % (uint64_t)g->K)) % g->K);
    const int h = std::min(head, left);
    if (h > 0) {
      afqmc_status s = group_segment(g, h, st);
      if (s != AFQMC_OK) return s;
      left -= h;
      t += (uint64_t)h;
    }
  }
  while (left >= g->K) {
    if (use_graph) {
      if (!g->exec) {
        AFQ_CK(hipStreamBeginCapture(g->cap, hipStreamCaptureModeThreadLocal));
        afqmc_status s = group_segment(g, g->K, g->cap);
        hipGraph_t gr = nullptr;
        const hipError_t ec = hipStreamEndCapture(g->cap, &gr);
        if (s != AFQMC_OK) {
          if (gr) (void)hipGraphDestroy(gr);
          return s;
        }
        AFQ_CK(ec);
        g->graph = gr;
        AFQ_CK(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
      }
      AFQ_CK(hipGraphLaunch(g->exec, st));
    } else {
      afqmc_status s = group_segment(g, g->K, st);
      if (s != AFQMC_OK) return s;
    }
    left -= g->K;
    t += (uint64_t)g->K;
  }
  if (left > 0) {
    afqmc_status s = group_segment(g, left, st);
    if (s != AFQMC_OK) return s;
  }
  return AFQMC_OK;
}

afqmc_status group_shape(afqmc_group* g, int threads, int K) {
  if (threads < 64 || threads > 512 || threads % 64) return fail(AFQMC_ERR_ARG, "threads: 64..512, multiple of 64");
  if (K < 1 || K > 1024) return fail(AFQMC_ERR_ARG, "segment steps: 1..1024");
  if (g->k_fixed && K != g->K) return fail(AFQMC_ERR_ARG, "segment steps are fixed by the combs");
  if (K > g->wsum_K) {
    void* p = nullptr;
    AFQ_CK(g->arena.alloc(&p, (size_t)K * g->w_total * 2 * sizeof(double)));
    g->wsum = (double*)p;
    g->wsum_K = K;
  }
  if (threads != g->threads || K != g->K) group_drop_graph(g);
  g->threads = threads;
  g->K = K;
  return AFQMC_OK;
}

}  // namespace

extern "C" {

afqmc_status afqmc_tune_cache_path(const char* path) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_path = path ? path : "";
  g_tune_path_set = true;
  return AFQMC_OK;
}

afqmc_status afqmc_resident_supported(const afqmc_trial* trial, int* ok) {
  if (!trial || !ok) return fail(AFQMC_ERR_ARG, "NULL trial / ok");
  *ok = resident_check(trial, nullptr, nullptr) == AFQMC_OK ? 1 : 0;
  return AFQMC_OK;
}

afqmc_status afqmc_group_create(afqmc_group** out, int n, const afqmc_group_member* mem,
                                void* stream) {
  if (!out || !mem || n < 1 || n > afq::kResMaxMembers)
    return fail(AFQMC_ERR_ARG, "group: out, members and 1 <= n <= 64 required");
  *out = nullptr;
  int device = -1;
  size_t lds = 0;
  for (int m = 0; m < n; ++m) {
    const afqmc_group_member& x = mem[m];
    if (!x.ham || !x.trial || !x.walkers) return fail(AFQMC_ERR_ARG, "group member with a NULL object");
    if (x.trial->ham != x.ham) return fail(AFQMC_ERR_STATE, "trial was built on another Hamiltonian");
    if (device >= 0 && x.ham->device != device) return fail(AFQMC_ERR_ARG, "group members on several devices");
    device = x.ham->device;
    afqmc_status s = check_walkers(x.trial, x.walkers);
    if (s != AFQMC_OK) return s;
    const afqmc_options& o = x.opt;
    if (!(x.dt > 0.0) || !std::isfinite(x.dt)) return fail(AFQMC_ERR_ARG, "dt must be positive");
    if (o.taylor_order < 1 || o.taylor_order > 64) return fail(AFQMC_ERR_ARG, "taylor_order");
    if (o.ortho_every < 0 || o.pc_every < 0) return fail(AFQMC_ERR_ARG, "negative interval");
    if (!std::isfinite(o.e_trial)) return fail(AFQMC_ERR_ARG, "e_trial is not finite");
    size_t l = 0;
    s = resident_check(x.trial, &o, &l);
    if (s != AFQMC_OK) return s;
    lds = std::max(lds, l);
    for (int k = 0; k < m; ++k)
      if (mem[k].walkers->phi_re == x.walkers->phi_re || mem[k].walkers->workspace == x.walkers->workspace)
        return fail(AFQMC_ERR_ARG, "two group members share walker buffers");
  }
  AFQ_CK(hipSetDevice(device));
  hipStream_t st = (hipStream_t)stream;
  afqmc_group* g = new afqmc_group();
  g->device = device;
  g->n = n;
  g->members.assign(mem, mem + n);
  g->lds_bytes = lds;
  auto bad = [&](afqmc_status code, const std::string& what) {
    group_drop_graph(g);
    if (g->cap) (void)hipStreamDestroy(g->cap);
    g->arena.release();
    delete g;
    return fail(code, what);
  };
  int kg = 0;
  std::ostringstream sig;
  {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) sig << prop.gcnArchName;
  }
  sig << ";resident";
  std::vector<std::string> shapes;
  for (int m = 0; m < n; ++m) {
    const afqmc_group_member& x = mem[m];
    afqmc_trial* tr = x.trial;
    afqmc_ham* hm = x.ham;
    afqmc_status err = AFQMC_OK;
    B1Entry* b1 = get_b1(tr, x.dt, st, &err);
    if (!b1) return bad(err, g_err);
    const int W = x.walkers->n_walkers;
    const WS ws = layout(tr, W, x.walkers->workspace);
    afq::ResMember r;
    std::memset(&r, 0, sizeof r);
    r.M = hm->M;
    r.Nt = tr->Nt;
    r.n0 = tr->nel[0];
    r.n1 = tr->nel[1];
    r.G = hm->G;
    r.W = W;
    r.wbase = g->w_total;
    r.system_id = x.walkers->system_id;
    r.ortho_every = x.opt.ortho_every;
    r.pc_every = x.opt.pc_every;
    r.MP4 = tr->MP4;
    r.NP0 = tr->NP[0];
    r.NP1 = tr->NP[1];
    r.order = x.opt.taylor_order;
    r.seed = x.seed;
    r.dt = x.dt;
    r.sqdt = std::sqrt(x.dt);
    r.e_trial = x.opt.e_trial;
    r.e_core = hm->e_core;
    r.ref_ls_re = tr->ref_ls[0];
    r.ref_ls_im = tr->ref_ls[1];
    r.ref_el_re = tr->ref_el[0];
    r.ref_el_im = tr->ref_el[1];
    r.L = hm->L;
    r.B1m = b1->d64;
    r.D0 = tr->D0;
    r.Lt0 = tr->Lt64[0];
    r.Lt1 = tr->Lt64[1];
    r.ht0 = tr->htil[0];
    r.ht1 = tr->htil[1];
    r.lbar = tr->lbar;
    r.vref_re = tr->vref_re;
    r.vref_im = tr->vref_im;
    r.phi_re = x.walkers->phi_re;
    r.phi_im = x.walkers->phi_im;
    r.weight = x.walkers->weight;
    r.ls_re = x.walkers->logovlp_re;
    r.ls_im = x.walkers->logovlp_im;
    r.el_re = x.walkers->eloc_re;
    r.el_im = x.walkers->eloc_im;
    r.v_re = ws.v_re;
    r.v_im = ws.v_im;
    void *ps = nullptr, *pp = nullptr, *pc = nullptr, *pn = nullptr;
    const size_t row = 2 * (size_t)r.M * r.Nt + 4 + 2 * (size_t)r.G;
    if (g->arena.alloc(&pn, 2 * sizeof(double)) ||
        (r.pc_every > 0 && (g->arena.alloc(&ps, (size_t)W * row * sizeof(double)) ||
                            g->arena.alloc(&pp, (size_t)W * sizeof(int)) ||
                            g->arena.alloc(&pc, (size_t)W * sizeof(double)))))
      return bad(AFQMC_ERR_OOM, "group allocation failed");
    r.snap = (double*)ps;
    r.parent = (int*)pp;
    r.cbuf = (double*)pc;
    r.comb_scal = (double*)pn;
    if (hipMemsetAsync(pn, 0, 2 * sizeof(double), st) != hipSuccess)
      return bad(AFQMC_ERR_DEVICE, "memset");
    g->h_mem.push_back(r);
    g->w_total += W;
    g->w_max = std::max(g->w_max, W);
    if (r.pc_every > 0) kg = std::gcd(kg, r.pc_every);
    std::ostringstream s1;
    s1 << r.M << "," << r.Nt << "," << r.G << "," << W << "," << r.order;
    shapes.push_back(s1.str());
  }
  std::sort(shapes.begin(), shapes.end());
  for (const auto& s1 : shapes) sig << "|" << s1;
  g->k_fixed = kg > 0;
  g->K = kg > 0 ? kg : 20;
  sig << ";segment=" << (kg > 0 ? std::to_string(kg) : std::string("free"));
  g->signature = sig.str();
  void *pm = nullptr, *pt = nullptr;
  if (g->arena.alloc(&pm, (size_t)n * sizeof(afq::ResMember)) || g->arena.alloc(&pt, 256))
    return bad(AFQMC_ERR_OOM, "group allocation failed");
  g->d_mem = (afq::ResMember*)pm;
  g->tdev = (uint64_t*)pt;
  if (hipMemcpyAsync(g->d_mem, g->h_mem.data(), (size_t)n * sizeof(afq::ResMember),
                     hipMemcpyHostToDevice, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return bad(AFQMC_ERR_DEVICE, "group table upload");
  if (hipStreamCreate(&g->cap) != hipSuccess) return bad(AFQMC_ERR_DEVICE, "capture stream");
  // launch shape: the tuning cache's entry for this signature, else 256 threads
  int thr = 256, K = g->K;
  const std::string path = tune_path();
  if (!path.empty()) {
    const auto all = tune_read(path);
    const auto it = all.find(g->signature);
    if (it != all.end() && (!g->k_fixed || it->second.segment == g->K)) {
      thr = it->second.threads;
      K = it->second.segment;
      g->tuned = 2;
    }
  }
  g->threads = 0;
  if (group_shape(g, thr, K) != AFQMC_OK) {
    g->tuned = 0;
    if (group_shape(g, 256, g->K) != AFQMC_OK) return bad(AFQMC_ERR_OOM, g_err);
  }
  *out = g;
  return AFQMC_OK;
}

afqmc_status afqmc_group_propagate(afqmc_group* g, int n_steps, uint64_t step0,
                                  double* const* emix_dev, void* stream) {
  if (!g) return fail(AFQMC_ERR_ARG, "NULL group");
  if (n_steps < 0) return fail(AFQMC_ERR_ARG, "n_steps must be >= 0");
  AFQ_CK(hipSetDevice(g->device));
  return group_run(g, n_steps, step0, emix_dev, (hipStream_t)stream, !g->timing);
}

afqmc_status afqmc_group_timing(afqmc_group* g, int enable) {
  if (!g) return fail(AFQMC_ERR_ARG, "NULL group");
  g->timing = enable != 0;
  g->timer.mask = g->timing ? 1u : 0u;
  if (g->timing) g->timer.reserve(512);
  return AFQMC_OK;
}

afqmc_status afqmc_group_timing_read(afqmc_group* g, int64_t* launches, int64_t* steps,
                                     double* total_ms) {
  if (!g || !launches || !steps || !total_ms) return fail(AFQMC_ERR_ARG, "NULL argument");
  AFQ_CK(hipSetDevice(g->device));
  AFQ_CK(g->timer.drain());
  *launches = g->timer.count[0];
  *total_ms = g->timer.total_ms[0];
  *steps = g->timed_steps;
  g->timer.count[0] = 0;
  g->timer.total_ms[0] = 0.0;
  g->timed_steps = 0;
  return AFQMC_OK;
}

afqmc_status afqmc_group_config(const afqmc_group* g, int* threads, int* segment_steps, int* tuned) {
  if (!g) return fail(AFQMC_ERR_ARG, "NULL group");
  if (threads) *threads = g->threads;
  if (segment_steps) *segment_steps = g->K;
  if (tuned) *tuned = g->tuned;
  return AFQMC_OK;
}

afqmc_status afqmc_group_set_config(afqmc_group* g, int threads, int segment_steps) {
  if (!g) return fail(AFQMC_ERR_ARG, "NULL group");
  AFQ_CK(hipSetDevice(g->device));
  afqmc_status s = group_shape(g, threads, segment_steps);
  if (s == AFQMC_OK) g->tuned = 0;
  return s;
}

afqmc_status afqmc_group_tune(afqmc_group* g, int steps, double* us_per_step, void* stream) {
  if (!g) return fail(AFQMC_ERR_ARG, "NULL group");
  if (steps < 1) return fail(AFQMC_ERR_ARG, "steps must be >= 1");
  AFQ_CK(hipSetDevice(g->device));
  hipStream_t st = (hipStream_t)stream;
  // save every member's walker state; candidates all run the same steps from it
  struct Saved { double* p; const double* src; size_t n; };
  std::vector<Saved> saved;
  Arena tmp;
  for (const afq::ResMember& r : g->h_mem) {
    const size_t mn = (size_t)r.W * r.M * r.Nt, wg = (size_t)r.W * r.G;
    const std::pair<const double*, size_t> bufs[] = {
        {r.phi_re, mn}, {r.phi_im, mn}, {r.weight, (size_t)r.W}, {r.ls_re, (size_t)r.W},
        {r.ls_im, (size_t)r.W}, {r.el_re, (size_t)r.W}, {r.el_im, (size_t)r.W}, {r.v_re, wg},
        {r.v_im, wg}};
    for (const auto& b : bufs) {
      if (b.second == 0) continue;
      void* p = nullptr;
      if (tmp.alloc(&p, b.second * sizeof(double)) != hipSuccess) {
        tmp.release();
        return fail(AFQMC_ERR_OOM, "tuning snapshot");
      }
      saved.push_back({(double*)p, b.first, b.second});
      if (hipMemcpyAsync(p, b.first, b.second * 8, hipMemcpyDeviceToDevice, st) != hipSuccess) {
        tmp.release();
        return fail(AFQMC_ERR_DEVICE, "tuning snapshot copy");
      }
    }
  }
  auto restore = [&]() -> hipError_t {
    for (const Saved& s : saved) {
      const hipError_t e = hipMemcpyAsync((void*)s.src, s.p, s.n * 8, hipMemcpyDeviceToDevice, st);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  };
  const int thr_c[] = {64, 128, 256, 512};
  std::vector<int> k_c;
  if (g->k_fixed) k_c.push_back(g->K);
  else k_c = {10, 20, 50};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    tmp.release();
    return fail(AFQMC_ERR_DEVICE, "tuning events");
  }
  double best = std::numeric_limits<double>::infinity();
  int bt = g->threads, bk = g->K;
  afqmc_status s = AFQMC_OK;
  for (int K : k_c)
    for (int thr : thr_c) {
      s = group_shape(g, thr, K);
      if (s != AFQMC_OK) break;
      const int n = std::max(steps, 2 * K);
      // one untimed pass (graph capture, caches), then the timed one
      for (int pass = 0; pass < 2 && s == AFQMC_OK; ++pass) {
        if (restore() != hipSuccess) { s = fail(AFQMC_ERR_DEVICE, "tuning restore"); break; }
        if (pass == 1 && hipEventRecord(e0, st) != hipSuccess) { s = fail(AFQMC_ERR_DEVICE, "event"); break; }
        s = group_run(g, n, 0, nullptr, st, true);
        if (pass == 1 && s == AFQMC_OK) {
          float ms = 0.f;
          if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
              hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            s = fail(AFQMC_ERR_DEVICE, "tuning timing");
            break;
          }
          const double us = 1e3 * ms / n;
          if (us < best) { best = us; bt = thr; bk = K; }
        }
      }
      if (s != AFQMC_OK) break;
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  const hipError_t re = restore();
  const hipError_t se = hipStreamSynchronize(st);
  tmp.release();
  if (s != AFQMC_OK) return s;
  if (re != hipSuccess || se != hipSuccess) return fail(AFQMC_ERR_DEVICE, "tuning restore");
  s = group_shape(g, bt, bk);
  if (s != AFQMC_OK) return s;
  g->tuned = 1;
  if (us_per_step) *us_per_step = best;
  const std::string path = tune_path();
  if (!path.empty()) tune_write(path, g->signature, TuneEntry{bt, bk, best});
  return AFQMC_OK;
}

void afqmc_free_group(afqmc_group* g) {
  if (!g) return;
  (void)hipSetDevice(g->device);
  group_drop_graph(g);
  if (g->cap) (void)hipStreamDestroy(g->cap);
  g->arena.release();
  delete g;
}

}  // extern "C"
