// Multi-determinant trial on gfx950 (arXiv 1804.03310, Sec. III).
//
// Psi_T = sum_i c_i |D_i>, where D_i is the reference D_0 with E_i <= 2 hole
// orbitals per spin replaced in place by particle orbitals.  With the
// reference overlap A = D_0^T phi, Theta_0 = phi A^-1 and Ghat = C^T Theta_0
// (all M orbitals; its top N x N block is the identity), the determinant
// lemma det(A + U V^T) = det(I + V^T A^-1 U) det(A) gives every overlap ratio
// as a small determinant of Ghat entries:
//     <D_i|phi> / <D_0|phi> = det(Ghat[particles, holes]).
// The matrix elements of one-body operators O follow from the same identity
// applied to det(D_i^T (1 + tO) phi) = det(A) det(Ghat[occ_i] + t P[occ_i]),
// P = C^T O Theta_0: writing Ghat[occ_i] in (hole, other) blocks, the
// t-expansion of the Schur complement of the identity block gives the t^1
// and t^2 coefficients (one-body element and the two-body L_g^2 element)
// from the reference quantities X0 = P[0:N, :], X0^2, Ghat and P at the
// particle rows, with O(N) work per entry and no inverse of the E x E block,
// so zero ratios (a walker on the reference) need no special case.
#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"

namespace afq {

struct Cx {
  double r, i;
};
__device__ inline Cx cx(double r, double i) { return Cx{r, i}; }
__device__ inline Cx operator+(Cx a, Cx b) { return Cx{a.r + b.r, a.i + b.i}; }
__device__ inline Cx operator-(Cx a, Cx b) { return Cx{a.r - b.r, a.i - b.i}; }
__device__ inline Cx operator*(Cx a, Cx b) { return Cx{a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__device__ inline Cx operator*(double s, Cx a) { return Cx{s * a.r, s * a.i}; }
__device__ inline Cx cdiv(Cx a, Cx b) {
  zdbl q = zdiv(zdbl{a.r, a.i}, zdbl{b.r, b.i});
  return Cx{q.re, q.im};
}

// det of the E x E block (E = 1, 2) and the mixed term m(X, Y) of
// det(X + tY) = det X + t m(X, Y) + t^2 det Y for 2 x 2.
__device__ inline Cx det2(const Cx X[2][2]) { return X[0][0] * X[1][1] - X[0][1] * X[1][0]; }
__device__ inline Cx mix2(const Cx X[2][2], const Cx Y[2][2]) {
  return X[0][0] * Y[1][1] + X[1][1] * Y[0][0] - X[0][1] * Y[1][0] - X[1][0] * Y[0][1];
}

// ===========================================================================
// Overlap ratios (FP64).  One block per walker.
// ===========================================================================
__global__ __launch_bounds__(256) void k_md_overlap(MDParams p, const double* __restrict__ thr,
                                                    const double* __restrict__ thi,
                                                    const double* ld_re, const double* ld_im,
                                                    double* c0_re, double* c0_im, double* tot_re,
                                                    double* tot_im, double* lsn_re, double* lsn_im) {
  extern __shared__ double gh[];  // per spin: Ghat [M][N] re then im
  __shared__ double red[4];
  const int w = blockIdx.x;
  const int M = p.M, Nt = p.Nt;
  const long wb = (long)w * M * Nt;
  double* g[2];
  g[0] = gh;
  g[1] = gh + 2 * M * p.sp[0].N;
  for (int s = 0; s < 2; ++s) {
    const int N = p.sp[s].N, off = p.sp[s].off;
    const double* C = p.sp[s].C;
    for (int e = threadIdx.x; e < M * N; e += blockDim.x) {
      const int q = e / N, b = e % N;
      double sr = 0.0, si = 0.0;
      for (int m = 0; m < M; ++m) {
        const double c = C[(long)m * M + q];
        sr += c * thr[wb + (long)m * Nt + off + b];
        si += c * thi[wb + (long)m * Nt + off + b];
      }
      g[s][e] = sr;
      g[s][M * N + e] = si;
    }
  }
  __syncthreads();
  double tr = 0.0, ti = 0.0;
  for (int i = threadIdx.x; i < p.n_det; i += blockDim.x) {
    Cx c0[2];
    for (int s = 0; s < 2; ++s) {
      const int N = p.sp[s].N;
      const int* ex = p.exc + (i * 2 + s) * 5;
      const int E = ex[0];
      const double* gr = g[s];
      const double* gi = g[s] + M * N;
      if (E == 0) {
        c0[s] = cx(1.0, 0.0);
      } else if (E == 1) {
        c0[s] = cx(gr[ex[3] * N + ex[1]], gi[ex[3] * N + ex[1]]);
      } else {
        Cx S[2][2];
        for (int a = 0; a < 2; ++a)
          for (int b = 0; b < 2; ++b)
            S[a][b] = cx(gr[ex[3 + a] * N + ex[1 + b]], gi[ex[3 + a] * N + ex[1 + b]]);
        c0[s] = det2(S);
      }
      c0_re[((long)w * 2 + s) * p.n_det + i] = c0[s].r;
      c0_im[((long)w * 2 + s) * p.n_det + i] = c0[s].i;
    }
    const Cx t = p.coeff[i] * (c0[0] * c0[1]);
    tr += t.r;
    ti += t.i;
  }
  tr = block_sum(tr, red);
  ti = block_sum(ti, red);
  if (threadIdx.x == 0) {
    tot_re[w] = tr;
    tot_im[w] = ti;
    const zdbl lg = zlog(zdbl{tr, ti});
    lsn_re[w] = ld_re[2 * w] + ld_re[2 * w + 1] + lg.re;
    lsn_im[w] = ld_im[2 * w] + ld_im[2 * w + 1] + lg.im;
  }
}

hipError_t md_overlap(hipStream_t st, int W, const MDParams& p, const double* thr,
                      const double* thi, const double* ld_re, const double* ld_im,
                      double* c0_re, double* c0_im, double* tot_re, double* tot_im,
                      double* lsn_re, double* lsn_im, size_t max_lds) {
  const size_t lds = (size_t)2 * p.M * (p.sp[0].N + p.sp[1].N) * sizeof(double);
  if (lds > max_lds) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_md_overlap, dim3(W), dim3(256), lds, st, p, thr, thi, ld_re, ld_im, c0_re,
                     c0_im, tot_re, tot_im, lsn_re, lsn_im);
  return hipGetLastError();
}

// ===========================================================================
// Energy and force bias.  One block per walker, both spins; loop over the
// Cholesky index g (g = G is the one-body h).  Per g and spin:
// P = C^T L_g Theta_0 (M x N) by 16x16x4 MFMA tiles in the contraction type
// (A operand (L_g C)[m][p] from global memory, B operand Theta_0 staged in
// LDS), X0 = P[0:N,:] and X0^2 in LDS, then every determinant's t^1 / t^2
// coefficients.  Per determinant the two-body numerator accumulates
// sum_g [c2_up c0_dn + c1_up c1_dn + c0_up c2_dn]; the force-bias numerator
// sum_i c_i (c1_up c0_dn + c0_up c1_dn) is reduced over determinants per g.
// ===========================================================================
template <typename T>
struct MdLds {
  T* tb[2];   // Theta_0 per spin, [MP4][NP] re then im
  T* gt[2];   // Ghat per spin, [M][N] re then im
  T* pb;      // P, [M][Nmax] re then im
  double* x2; // X0^2, [Nmax][Nmax] re then im
  double* scal;
};

// t^1 and t^2 coefficients of det(Ghat[occ] + t P[occ]) for one determinant
// and spin (relative to det A), from its (e, f) entries (e over particles v_e,
// f over holes r_f): S0 = Ghat[v_e][r_f], Q = P[v_e][r_f], GX = (Ghat X0)[v_e][r_f],
// PX = (P X0)[v_e][r_f], GXX = (Ghat X0^2)[v_e][r_f], XR = X0[r_e][r_f] and
// X2R = X0^2[r_e][r_f].  E (the excitation rank, 1 or 2) is a template
// parameter so that every small E x E array lives in registers.
template <int E>
__device__ inline void md_det_algebra(const Cx (&S0)[2][2], const Cx (&Q)[2][2],
                                      const Cx (&GX)[2][2], const Cx (&PX)[2][2],
                                      const Cx (&GXX)[2][2], const Cx (&XR)[2][2],
                                      const Cx (&X2R)[2][2], Cx trx0, Cx trx2, Cx& c1, Cx& c2) {
  const Cx e2 = 0.5 * (trx0 * trx0 - trx2);
  Cx S1[2][2], S2[2][2];
#pragma unroll
  for (int e = 0; e < E; ++e)
#pragma unroll
    for (int f = 0; f < E; ++f) {
      Cx bq = GX[e][f], qq = PX[e][f], gxx = GXX[e][f];
#pragma unroll
      for (int g = 0; g < E; ++g) {
        bq = bq - S0[e][g] * XR[g][f];
        qq = qq - Q[e][g] * XR[g][f];
        gxx = gxx - S0[e][g] * X2R[g][f];
      }
      S1[e][f] = Q[e][f] - bq;
      Cx bqq = gxx;
      // U_R X0[R,R] with U_R = bq (row e)
#pragma unroll
      for (int g = 0; g < E; ++g) {
        Cx ueg = GX[e][g];
#pragma unroll
        for (int h = 0; h < E; ++h) ueg = ueg - S0[e][h] * XR[h][g];
        bqq = bqq - ueg * XR[g][f];
      }
      S2[e][f] = bqq - qq;
    }
  Cx t1 = trx0, touch = cx(0, 0);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    t1 = t1 - XR[e][e];
    touch = touch + (XR[e][e] * trx0 - X2R[e][e]);
  }
  if (E == 2) touch = touch - (XR[0][0] * XR[1][1] - XR[0][1] * XR[1][0]);
  const Cx t2 = e2 - touch;
  Cx d0, d1, d2;
  if (E == 1) {
    d0 = S0[0][0];
    d1 = S1[0][0];
    d2 = S2[0][0];
  } else {
    d0 = det2(S0);
    d1 = mix2(S0, S1);
    d2 = det2(S1) + mix2(S0, S2);
  }
  c1 = d1 + t1 * d0;
  c2 = d2 + t1 * d1 + t2 * d0;
}

// The same from the full-row reference quantities in LDS (holes h0, h1 and
// particles v0, v1 as orbital indices), the sums over the occupied index
// taken here.
template <int E, typename T>
__device__ inline void md_det_coeffs_e(int N, int Nmax, int h0, int h1, int v0, int v1,
                                       const T* gr, const T* gi, const T* pr, const T* pi,
                                       const double* x2r, const double* x2i, Cx trx0, Cx trx2,
                                       Cx& c1, Cx& c2) {
  const int hole[2] = {h0, h1}, part[2] = {v0, v1};
  auto X0 = [&](int a, int b) { return cx((double)pr[a * Nmax + b], (double)pi[a * Nmax + b]); };
  auto X2 = [&](int a, int b) { return cx(x2r[a * Nmax + b], x2i[a * Nmax + b]); };
  auto Gv = [&](int v, int c) { return cx((double)gr[v * N + c], (double)gi[v * N + c]); };
  Cx S0[2][2], Q[2][2], GX[2][2], PX[2][2], GXX[2][2], XR[2][2], X2R[2][2];
#pragma unroll
  for (int e = 0; e < E; ++e)
#pragma unroll
    for (int f = 0; f < E; ++f) {
      const int v = part[e], r = hole[f];
      S0[e][f] = Gv(v, r);
      Q[e][f] = X0(v, r);
      Cx gx = cx(0, 0), px = cx(0, 0), gxx = cx(0, 0);
      for (int c = 0; c < N; ++c) {
        const Cx g = Gv(v, c), pc = X0(v, c), xcr = X0(c, r);
        gx = gx + g * xcr;
        px = px + pc * xcr;
        gxx = gxx + g * X2(c, r);
      }
      GX[e][f] = gx;
      PX[e][f] = px;
      GXX[e][f] = gxx;
      XR[e][f] = X0(hole[e], r);
      X2R[e][f] = X2(hole[e], r);
    }
  md_det_algebra<E>(S0, Q, GX, PX, GXX, XR, X2R, trx0, trx2, c1, c2);
}

template <typename T>
__device__ inline void md_det_coeffs(int N, int Nmax, int E, int h0, int h1, int v0, int v1,
                                     const T* gr, const T* gi, const T* pr, const T* pi,
                                     const double* x2r, const double* x2i, Cx trx0, Cx trx2,
                                     Cx& c1, Cx& c2) {
  if (E == 0) {
    c1 = trx0;
    c2 = 0.5 * (trx0 * trx0 - trx2);
  } else if (E == 1) {
    md_det_coeffs_e<1>(N, Nmax, h0, h1, v0, v1, gr, gi, pr, pi, x2r, x2i, trx0, trx2, c1, c2);
  } else {
    md_det_coeffs_e<2>(N, Nmax, h0, h1, v0, v1, gr, gi, pr, pi, x2r, x2i, trx0, trx2, c1, c2);
  }
}

template <typename T, int DPT>
__global__ __launch_bounds__(256) void k_md_energy(MDParams p, int Nmax, int NPmax,
                                                   const double* __restrict__ thr,
                                                   const double* __restrict__ thi,
                                                   const double* __restrict__ c0_re,
                                                   const double* __restrict__ c0_im,
                                                   const double* tot_re, const double* tot_im,
                                                   double* v_re, double* v_im, double* eln_re,
                                                   double* eln_im, int* vfin) {
  extern __shared__ unsigned char lds_raw[];
  __shared__ double red[4];
  __shared__ double scal[4];
  typedef Mfma<T> MM;
  typedef typename MM::acc_t acc_t;
  const int w = blockIdx.x;
  const int M = p.M, Nt = p.Nt, G = p.G, MP4 = p.MP4;
  const long wb = (long)w * M * Nt;
  const int wv = wave_id(), l = lane_id(), li = l & 15, lk = l >> 4;
  // LDS carve-up
  T* base = (T*)lds_raw;
  T* tb[2];
  T* gt[2];
  tb[0] = base;
  tb[1] = tb[0] + 2 * MP4 * NPmax;
  gt[0] = tb[1] + 2 * MP4 * NPmax;
  gt[1] = gt[0] + 2 * M * Nmax;
  T* pb = gt[1] + 2 * M * Nmax;
  double* x2 = (double*)(pb + 2 * M * Nmax + ((2 * M * Nmax * sizeof(T)) % 8 ? 1 : 0));
  // stage Theta_0 (B operand, zero padded) and Ghat = C^T Theta_0 in T
  for (int s = 0; s < 2; ++s) {
    const int N = p.sp[s].N, off = p.sp[s].off;
    for (int e = threadIdx.x; e < MP4 * NPmax; e += blockDim.x) {
      const int m = e / NPmax, b = e % NPmax;
      const bool ok = m < M && b < N;
      tb[s][e] = ok ? (T)thr[wb + (long)m * Nt + off + b] : (T)0;
      tb[s][MP4 * NPmax + e] = ok ? (T)thi[wb + (long)m * Nt + off + b] : (T)0;
    }
    const double* C = p.sp[s].C;
    for (int e = threadIdx.x; e < M * N; e += blockDim.x) {
      const int q = e / N, b = e % N;
      double sr = 0.0, si = 0.0;
      for (int m = 0; m < M; ++m) {
        const double c = C[(long)m * M + q];
        sr += c * thr[wb + (long)m * Nt + off + b];
        si += c * thi[wb + (long)m * Nt + off + b];
      }
      gt[s][q * N + b] = (T)sr;
      gt[s][M * N + q * N + b] = (T)si;
    }
  }
  // per-determinant state
  const Cx tot = cx(tot_re[w], tot_im[w]);
  int myE[DPT][2], myH[DPT][2][2], myP[DPT][2][2];
  Cx c0u[DPT], c0d[DPT], a2u[DPT], a2d[DPT], a11[DPT], c1h[DPT][2];
  double coef[DPT];
#pragma unroll
  for (int k = 0; k < DPT; ++k) {
    const int i = threadIdx.x + k * blockDim.x;
    const bool ok = i < p.n_det;
    coef[k] = ok ? p.coeff[i] : 0.0;
    for (int s = 0; s < 2; ++s) {
      const int* ex = p.exc + ((ok ? i : 0) * 2 + s) * 5;
      myE[k][s] = ok ? ex[0] : 0;
      myH[k][s][0] = ex[1];
      myH[k][s][1] = ex[2];
      myP[k][s][0] = ex[3];
      myP[k][s][1] = ex[4];
    }
    c0u[k] = ok ? cx(c0_re[((long)w * 2) * p.n_det + i], c0_im[((long)w * 2) * p.n_det + i]) : cx(0, 0);
    c0d[k] = ok ? cx(c0_re[((long)w * 2 + 1) * p.n_det + i], c0_im[((long)w * 2 + 1) * p.n_det + i]) : cx(0, 0);
    a2u[k] = a2d[k] = a11[k] = cx(0, 0);
    c1h[k][0] = c1h[k][1] = cx(0, 0);
  }
  int fin = 1;
  __syncthreads();
  for (int g = 0; g <= G; ++g) {
    Cx c1[DPT][2], c2[DPT][2];
    for (int s = 0; s < 2; ++s) {
      const int N = p.sp[s].N;
      if (N == 0) {
#pragma unroll
        for (int k = 0; k < DPT; ++k) {
          if (s) { c1[k][1] = cx(0, 0); c2[k][1] = cx(0, 0); }
          else { c1[k][0] = cx(0, 0); c2[k][0] = cx(0, 0); }
        }
        continue;
      }
      // P = (L_g C)^T Theta_0: rows p < M, columns b < N
      const T* __restrict__ A = (const T*)p.sp[s].LC + (long)g * M * M;
      const int RT = (M + 15) / 16, CT = (N + 15) / 16, NTL = RT * CT;
      const T* tbs = s ? tb[1] : tb[0];
      // two output tiles of the wave at a time; the A fragments (L_g C, read
      // from L2 / the infinity cache) of both tiles for a batch of KB k steps
      // are requested together before the first MFMA, so one memory latency
      // covers the batch (FP32: KB = 32 covers M <= 128 in one batch)
      constexpr int KB = sizeof(T) == 4 ? 32 : 16;
      const int KSt = MP4 / 4;
      for (int t0 = wv; t0 < NTL; t0 += 8) {
        const int t1 = t0 + 4;
        const bool has1 = t1 < NTL;
        const int rt0 = t0 / CT, ct0 = t0 % CT, rt1 = (has1 ? t1 : t0) / CT, ct1 = (has1 ? t1 : t0) % CT;
        // rows past M clamped to the last one (their results are never stored)
        const int prow0 = min(16 * rt0 + li, M - 1), prow1 = min(16 * rt1 + li, M - 1);
        acc_t ar0 = MM::zero(), ai0 = MM::zero(), ar1 = MM::zero(), ai1 = MM::zero();
        for (int kb = 0; kb < KSt; kb += KB) {
          T a0[KB], a1[KB];
#pragma unroll
          for (int j = 0; j < KB; ++j) {
            const int m = min(4 * (kb + j) + lk, M - 1);
            const bool ok = kb + j < KSt && 4 * (kb + j) + lk < M;
            const T x0 = A[(long)m * M + prow0];
            const T x1 = A[(long)m * M + prow1];
            a0[j] = ok ? x0 : (T)0;
            a1[j] = ok ? x1 : (T)0;
          }
#pragma unroll
          for (int j = 0; j < KB; ++j) {
            if (kb + j < KSt) {
              const int m = 4 * (kb + j) + lk;
              const T br0 = tbs[m * NPmax + 16 * ct0 + li];
              const T bi0 = tbs[MP4 * NPmax + m * NPmax + 16 * ct0 + li];
              const T br1 = tbs[m * NPmax + 16 * ct1 + li];
              const T bi1 = tbs[MP4 * NPmax + m * NPmax + 16 * ct1 + li];
              ar0 = MM::mma(a0[j], br0, ar0);
              ai0 = MM::mma(a0[j], bi0, ai0);
              ar1 = MM::mma(a1[j], br1, ar1);
              ai1 = MM::mma(a1[j], bi1, ai1);
            }
          }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r0 = 16 * rt0 + MM::row(lk, v), c0 = 16 * ct0 + li;
          if (r0 < M && c0 < N) {
            pb[r0 * Nmax + c0] = (T)ar0[v];
            pb[M * Nmax + r0 * Nmax + c0] = (T)ai0[v];
          }
          const int r1 = 16 * rt1 + MM::row(lk, v), c1 = 16 * ct1 + li;
          if (has1 && r1 < M && c1 < N) {
            pb[r1 * Nmax + c1] = (T)ar1[v];
            pb[M * Nmax + r1 * Nmax + c1] = (T)ai1[v];
          }
        }
      }
      __syncthreads();
      // X0^2 and the traces
      for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
        const int a = e / N, b = e % N;
        double sr = 0.0, si = 0.0;
        for (int c = 0; c < N; ++c) {
          const double xr = (double)pb[a * Nmax + c], xi = (double)pb[M * Nmax + a * Nmax + c];
          const double yr = (double)pb[c * Nmax + b], yi = (double)pb[M * Nmax + c * Nmax + b];
          sr += xr * yr - xi * yi;
          si += xr * yi + xi * yr;
        }
        x2[a * Nmax + b] = sr;
        x2[Nmax * Nmax + a * Nmax + b] = si;
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        double t0r = 0, t0i = 0, t2r = 0, t2i = 0;
        for (int a = 0; a < N; ++a) {
          t0r += (double)pb[a * Nmax + a];
          t0i += (double)pb[M * Nmax + a * Nmax + a];
          t2r += x2[a * Nmax + a];
          t2i += x2[Nmax * Nmax + a * Nmax + a];
        }
        scal[0] = t0r; scal[1] = t0i; scal[2] = t2r; scal[3] = t2i;
      }
      __syncthreads();
      const Cx trx0 = cx(scal[0], scal[1]), trx2 = cx(scal[2], scal[3]);
#pragma unroll
      for (int k = 0; k < DPT; ++k) {
        const int i = threadIdx.x + k * blockDim.x;
        // spin-indexed per-determinant values by select, so that no array is
        // indexed with the runtime spin (which would place it in scratch memory)
        Cx o1 = cx(0, 0), o2 = cx(0, 0);
        if (i < p.n_det) {
          const int E = s ? myE[k][1] : myE[k][0];
          const int h0 = s ? myH[k][1][0] : myH[k][0][0], h1 = s ? myH[k][1][1] : myH[k][0][1];
          const int v0 = s ? myP[k][1][0] : myP[k][0][0], v1 = s ? myP[k][1][1] : myP[k][0][1];
          const T* gs = s ? gt[1] : gt[0];
          md_det_coeffs<T>(N, Nmax, E, h0, h1, v0, v1, gs, gs + M * N, pb, pb + M * Nmax, x2,
                           x2 + Nmax * Nmax, trx0, trx2, o1, o2);
        }
        if (s) { c1[k][1] = o1; c2[k][1] = o2; } else { c1[k][0] = o1; c2[k][0] = o2; }
      }
      __syncthreads();
    }
    if (g < G) {
      double vr = 0.0, vi = 0.0;
#pragma unroll
      for (int k = 0; k < DPT; ++k) {
        a2u[k] = a2u[k] + c2[k][0];
        a2d[k] = a2d[k] + c2[k][1];
        a11[k] = a11[k] + c1[k][0] * c1[k][1];
        const Cx vn = coef[k] * (c1[k][0] * c0d[k] + c0u[k] * c1[k][1]);
        vr += vn.r;
        vi += vn.i;
      }
      vr = block_sum(vr, red);
      vi = block_sum(vi, red);
      if (threadIdx.x == 0) {
        const Cx v = cdiv(cx(vr, vi), tot);
        v_re[(long)w * G + g] = v.r;
        v_im[(long)w * G + g] = v.i;
        if (!isfinite(v.r) || !isfinite(v.i)) fin = 0;
      }
    } else {
#pragma unroll
      for (int k = 0; k < DPT; ++k) {
        c1h[k][0] = c1[k][0];
        c1h[k][1] = c1[k][1];
      }
    }
  }
  double nr = 0.0, ni = 0.0;
#pragma unroll
  for (int k = 0; k < DPT; ++k) {
    const Cx n = coef[k] * (p.e_core * (c0u[k] * c0d[k]) + c1h[k][0] * c0d[k] + c0u[k] * c1h[k][1] +
                            c0d[k] * a2u[k] + c0u[k] * a2d[k] + a11[k]);
    nr += n.r;
    ni += n.i;
  }
  nr = block_sum(nr, red);
  ni = block_sum(ni, red);
  if (threadIdx.x == 0) {
    const Cx e = cdiv(cx(nr, ni), tot);
    eln_re[w] = e.r;
    eln_im[w] = e.i;
    vfin[w] = fin;
  }
}

// ===========================================================================
// Energy and force bias, FP32 contractions over compact rows: four walkers per
// block and two wavefronts per walker, a producer and a consumer, so that the
// matrix-core work of one phase overlaps the vector work of the previous one.  Phases q = (slot, spin) run in the order slot G+1 (the rows of C:
// Ghat at the particle rows), then the operators 0..G.  In step tau:
//  - the producers form P(tau) = LCc[slot]^T Theta_0 for their walkers by
//    16x16x4 MFMA, the operator (FP32, M padded to 4 KS k rows, in MFMA
//    fragment order) staged in LDS once for the four walkers and Theta_0
//    held in registers as the B operand, into LDS buffer tau mod 2;
//  - each consumer works on P(tau - 1) of its walker: X0^2 (MFMA) and the
//    traces, the sums over the occupied index of every listed (particle,
//    hole) pair (the lane owning the particle, its Ghat row held in
//    registers) with the coefficients of the single excitation it defines,
//    and every other determinant's t^1 / t^2 coefficients, accumulated per
//    determinant in FP64.
// After a barrier the producers store the next operator (loaded into their
// registers a step earlier) and request the one after it; a second barrier
// publishes it.
// ===========================================================================
constexpr int kMdWalkers = 4;

struct MdRowsLds {
  int ns;      // row stride (elements) of P and X0^2
  int wbytes;  // bytes of one walker's region
  int pw0, pw1, x2, tab, e1, s0a, s0b;  // offsets inside a walker's region
  int wave0;   // offset of walker 0's region
  int total;
};

inline MdRowsLds md_rows_lds(const MDParams& p, int ks) {
  MdRowsLds o;
  auto al = [](long b) { return (int)((b + 15) & ~15L); };
  const int N0 = p.sp[0].N, N1 = p.sp[1].N, Nmax = N0 > N1 ? N0 : N1;
  const int R0 = p.rows.R[0], R1 = p.rows.R[1];
  const int rp = p.rows.RP[0] > p.rows.RP[1] ? p.rows.RP[0] : p.rows.RP[1];
  const int np = p.rows.npair[0] > p.rows.npair[1] ? p.rows.npair[0] : p.rows.npair[1];
  o.ns = Nmax > 0 ? Nmax : 1;
  const int pwb = al((long)(R0 > R1 ? R0 : R1) * o.ns * 8);
  int q = 0;
  o.pw0 = q;
  q += pwb;
  o.pw1 = q;
  q += pwb;
  o.x2 = q;
  q += al((long)Nmax * o.ns * 8);
  o.tab = q;
  q += al((long)np * 24);
  o.e1 = q;
  q += al((long)np * 32);
  o.s0a = q;
  q += al((long)p.rows.npair[0] * 8);
  o.s0b = q;
  q += al((long)p.rows.npair[1] * 8);
  o.wbytes = q;
  o.wave0 = al((long)4 * ks * rp * 4);  // the operator: 4 ks rows (k) x rp columns
  o.total = o.wave0 + kMdWalkers * o.wbytes;
  return o;
}

// One 16-row tile of P.  The operator is stored in MFMA fragment order:
// element (m, c) with m = 16 J + 4 jj + lk and c = 16 rt + li sits at float
// index (((J RTP + rt) 4 + lk) 16 + li) 4 + jj, so lane (li, lk) reads the A
// values of four k steps with one 128-bit load (`a4` points at J = 0 of the
// tile, `jstride` = RTP 64 vectors per J).  The sum over k alternates between
// two accumulators per part, so that consecutive MFMAs are independent.
template <int KS>
__device__ __forceinline__ void md_rows_tile(const afq_f4* __restrict__ a4, int jstride,
                                             const float (&br)[KS], const float (&bi)[KS],
                                             afq_f4& er, afq_f4& ei, afq_f4& orr, afq_f4& oi) {
  typedef Mfma<float> MM;
  afq_f4 an = a4[0];
#pragma unroll
  for (int J = 0; J < KS / 4; ++J) {
    // the next k block's load is issued before this block's MFMAs
    const afq_f4 a = an;
    if (J + 1 < KS / 4) an = a4[(J + 1) * jstride];
    er = MM::mma(a[0], br[4 * J], er);
    ei = MM::mma(a[0], bi[4 * J], ei);
    orr = MM::mma(a[1], br[4 * J + 1], orr);
    oi = MM::mma(a[1], bi[4 * J + 1], oi);
    er = MM::mma(a[2], br[4 * J + 2], er);
    ei = MM::mma(a[2], bi[4 * J + 2], ei);
    orr = MM::mma(a[3], br[4 * J + 3], orr);
    oi = MM::mma(a[3], bi[4 * J + 3], oi);
  }
}

// t^1 / t^2 coefficients of a single excitation r -> v (E = 1 of the algebra
// above) from its entries s = S0, q = Q, gx = GX, px = PX, gxx = GXX, x =
// X0[r][r], y = X0^2[r][r], Tr X0 and e2 = (Tr^2 X0 - Tr X0^2) / 2.
__device__ inline void md_single(Cx s, Cx q, Cx gx, Cx px, Cx gxx, Cx x, Cx y, Cx trx0, Cx e2,
                                 Cx& c1, Cx& c2) {
  const Cx bq = gx - s * x;
  const Cx s1 = q - bq;
  const Cx s2 = (gxx - s * y) - bq * x - (px - q * x);
  const Cx t1 = trx0 - x;
  const Cx t2 = e2 - (x * trx0 - y);
  c1 = s1 + t1 * s;
  c2 = s2 + t1 * s1 + t2 * s;
}

// One determinant's coefficients for one spin from the compact-row quantities
// of its walker: particles as compact indices t (row N + t of P), holes r,
// the pair sums (GX, PX, GXX) from the table and S0 = Ghat[v][r] from the
// set-up-time table of the pair.
template <int E>
__device__ inline void md_det_rows(int N, int NS, unsigned w0, unsigned w1, unsigned w2,
                                   const float2* pw, const float2* x2, const float2* tab,
                                   const float2* s0t, Cx trx0, Cx trx2, Cx& c1, Cx& c2) {
  const int hole[2] = {(int)((w0 >> 2) & 31u), (int)((w0 >> 7) & 31u)};
  const int part[2] = {(int)((w0 >> 12) & 255u), (int)((w0 >> 20) & 255u)};
  const int pidx[2][2] = {{(int)(w1 & 0xffffu), (int)(w1 >> 16)},
                          {(int)(w2 & 0xffffu), (int)(w2 >> 16)}};
  Cx S0[2][2], Q[2][2], GX[2][2], PX[2][2], GXX[2][2], XR[2][2], X2R[2][2];
#pragma unroll
  for (int e = 0; e < E; ++e)
#pragma unroll
    for (int f = 0; f < E; ++f) {
      const int k = pidx[e][f];
      const float2 g = s0t[k];
      const float2 q = pw[(N + part[e]) * NS + hole[f]];
      const float2 x = pw[hole[e] * NS + hole[f]];
      const float2 y = x2[hole[e] * NS + hole[f]];
      const float2* tb = tab + 3 * k;
      const float2 t0 = tb[0], t1 = tb[1], t2 = tb[2];
      S0[e][f] = cx(g.x, g.y);
      Q[e][f] = cx(q.x, q.y);
      XR[e][f] = cx(x.x, x.y);
      X2R[e][f] = cx(y.x, y.y);
      GX[e][f] = cx(t0.x, t0.y);
      PX[e][f] = cx(t1.x, t1.y);
      GXX[e][f] = cx(t2.x, t2.y);
    }
  md_det_algebra<E>(S0, Q, GX, PX, GXX, XR, X2R, trx0, trx2, c1, c2);
}

// Phase q of the compact-row kernel works on slot md_rows_slot(q, G) for
// spin q & 1: slot G+1 (the rows of C) first, then the operators 0..G.
__device__ __forceinline__ int md_rows_slot(int q, int G) { return q < 2 ? G + 1 : (q >> 1) - 1; }

// Loads phase q's operator (4 KS x RP floats in fragment order, contiguous)
// into the staging registers of the producer threads (256), 16 bytes per
// thread and register; every thread loads all of them (indices past the end
// are clamped; the set-up gives a spin without electrons a 16-float table) so
// that the array stays in registers.
template <int KS>
__device__ __forceinline__ void md_rows_issue(const MDParams& p, int G, int q, int tid,
                                              afq_f4 (&pf)[kMdRowsPF]) {
  const int s = q & 1, rp = s ? p.rows.RP[1] : p.rows.RP[0];
  const float* base = s ? p.rows.LCc[1] : p.rows.LCc[0];
  const int n4 = KS * rp;
  const int last = n4 > 0 ? n4 - 1 : 0;
  const afq_f4* src = (const afq_f4*)(base + (size_t)md_rows_slot(q, G) * 4 * KS * rp);
#pragma unroll
  for (int u = 0; u < kMdRowsPF; ++u) {
    const int e = tid + 256 * u;
    pf[u] = src[e < last ? e : last];
  }
}

// Stores the staging registers into the LDS operator buffer (same order).
template <int KS>
__device__ __forceinline__ void md_rows_stage(const MDParams& p, int q, int tid,
                                              const afq_f4 (&pf)[kMdRowsPF], afq_f4* abuf) {
  const int s = q & 1, rp = s ? p.rows.RP[1] : p.rows.RP[0];
  const int n4 = KS * rp;
#pragma unroll
  for (int u = 0; u < kMdRowsPF; ++u) {
    const int e = tid + 256 * u;
    if (e < n4) abuf[e] = pf[u];
  }
}

// Producer: Theta_0 as B fragments (lane (li, lk) holds row 4 j + lk, column
// li of each spin; zero past M and past N), then per step the product of the
// staged operator into the P buffer of the step.
template <int KS>
__device__ void md_rows_producer(const MDParams& p, const MdRowsLds& L, unsigned char* lds,
                                 int wl, long wb, const double* __restrict__ thr,
                                 const double* __restrict__ thi) {
  typedef Mfma<float> MM;
  typedef MM::acc_t acc_t;
  const int l = lane_id(), li = l & 15, lk = l >> 4;
  const int tid = 64 * (wave_id() >> 1) + l;  // 0 .. 255 over the four producers
  const int M = p.M, Nt = p.Nt, G = p.G, NS = L.ns, NPH = 2 * (G + 2);
  afq_f4* abuf = (afq_f4*)lds;
  unsigned char* reg = lds + L.wave0 + wl * L.wbytes;
  float b0r[KS], b0i[KS], b1r[KS], b1i[KS];
  {
    const int N0 = p.sp[0].N, N1 = p.sp[1].N, o1 = p.sp[1].off;
#pragma unroll
    for (int j = 0; j < KS; ++j) {
      const int m = 4 * j + lk;
      const long o = wb + (long)(m < M ? m : 0) * Nt;
      const bool ok0 = m < M && li < N0, ok1 = m < M && li < N1;
      const long i0 = o + (ok0 ? li : 0), i1 = o + (ok1 ? o1 + li : 0);
      b0r[j] = ok0 ? (float)thr[i0] : 0.f;
      b0i[j] = ok0 ? (float)thi[i0] : 0.f;
      b1r[j] = ok1 ? (float)thr[i1] : 0.f;
      b1i[j] = ok1 ? (float)thi[i1] : 0.f;
    }
  }
  afq_f4 pf[kMdRowsPF];
  md_rows_issue<KS>(p, G, 0, tid, pf);
  md_rows_stage<KS>(p, 0, tid, pf, abuf);
  md_rows_issue<KS>(p, G, 1, tid, pf);
  __syncthreads();
  for (int tau = 0; tau <= NPH; ++tau) {
    if (tau < NPH) {
      const int s = tau & 1;
      const int N = s ? p.sp[1].N : p.sp[0].N;
      const int R = s ? p.rows.R[1] : p.rows.R[0];
      const int RT = (R + 15) >> 4;
      const int RTP = (s ? p.rows.RP[1] : p.rows.RP[0]) >> 4;
      float2* pw = (float2*)(reg + ((tau & 1) ? L.pw1 : L.pw0));
      for (int rt = 0; rt < RT; ++rt) {
        acc_t er = MM::zero(), ei = MM::zero(), orr = MM::zero(), oi = MM::zero();
        const afq_f4* a4 = abuf + rt * 64 + l;
        if (s == 0)
          md_rows_tile<KS>(a4, RTP * 64, b0r, b0i, er, ei, orr, oi);
        else
          md_rows_tile<KS>(a4, RTP * 64, b1r, b1i, er, ei, orr, oi);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = 16 * rt + 4 * lk + v;
          if (li < N && row < R) pw[row * NS + li] = make_float2(er[v] + orr[v], ei[v] + oi[v]);
        }
      }
    }
    __syncthreads();  // P(tau) written; every producer is done with the operator
    if (tau + 1 < NPH) md_rows_stage<KS>(p, tau + 1, tid, pf, abuf);
    if (tau + 2 < NPH) md_rows_issue<KS>(p, G, tau + 2, tid, pf);
    __syncthreads();  // the next operator is in LDS
  }
}

// Consumer: the determinant algebra of phase tau - 1 in step tau.
template <int DPL>
__device__ void md_rows_consumer(const MDParams& p, const MdRowsLds& L, unsigned char* lds, int wl,
                                 int w, int wr, bool live, const double* __restrict__ c0_re,
                                 const double* __restrict__ c0_im, const double* tot_re,
                                 const double* tot_im, double* v_re, double* v_im, double* eln_re,
                                 double* eln_im, int* vfin) {
  const int l = lane_id();
  const int G = p.G, NS = L.ns, n_det = p.n_det, NPH = 2 * (G + 2);
  unsigned char* reg = lds + L.wave0 + wl * L.wbytes;
  float2* x2 = (float2*)(reg + L.x2);
  float2* tab = (float2*)(reg + L.tab);
  double2* e1t = (double2*)(reg + L.e1);
  float2* s0a = (float2*)(reg + L.s0a);
  float2* s0b = (float2*)(reg + L.s0b);
  // per-determinant state: slot i = l + 64 k holds determinant dx[i][6];
  // acc accumulates cd c2_up + cu c2_dn + coef c1_up c1_dn over the vectors,
  // plus cd c1_up + cu c1_dn for h and e_core coef c0_up c0_dn, with
  // cu = coef c0_up and cd = coef c0_dn
  unsigned dxw[DPL][2][3];
  double coef[DPL];
  Cx cu[DPL], cd[DPL], acc[DPL], c1p[DPL];
#pragma unroll
  for (int k = 0; k < DPL; ++k) {
    const int i = l + 64 * k;
    const bool ok = i < n_det;
    const int* dr = p.rows.dx + (ok ? i : 0) * kMdDx;
    const int ic = ok ? dr[6] : 0;
    coef[k] = ok ? p.coeff[ic] : 0.0;
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int q = 0; q < 3; ++q) dxw[k][s][q] = ok ? (unsigned)dr[s * 3 + q] : 0u;
    const long u = ((long)wr * 2) * n_det + ic, d = ((long)wr * 2 + 1) * n_det + ic;
    const Cx c0u = ok ? cx(c0_re[u], c0_im[u]) : cx(0, 0);
    const Cx c0d = ok ? cx(c0_re[d], c0_im[d]) : cx(0, 0);
    cu[k] = coef[k] * c0u;
    cd[k] = coef[k] * c0d;
    acc[k] = p.e_core * (cu[k] * c0d);
    c1p[k] = cx(0, 0);
  }
  const Cx tot = cx(tot_re[wr], tot_im[wr]);
  int fin = 1;
  // the Ghat row of particle t = l of each spin (FP32), owned by lane t
  float2 gh0[kMdRowsMaxN], gh1[kMdRowsMaxN];
#pragma unroll
  for (int c = 0; c < kMdRowsMaxN; ++c) gh0[c] = gh1[c] = make_float2(0.f, 0.f);
  __syncthreads();  // the producers' first operator is staged
  for (int tau = 0; tau <= NPH; ++tau) {
    if (tau >= 1) {
      const int q = tau - 1, s = q & 1, slot = md_rows_slot(q, G);
      const int N = s ? p.sp[1].N : p.sp[0].N;
      const int R = s ? p.rows.R[1] : p.rows.R[0];
      const int nv = R - N;
      const float2* pw = (const float2*)(reg + ((q & 1) ? L.pw1 : L.pw0));
      const int* pl = s ? p.rows.pair[1] : p.rows.pair[0];
      const int* pb = s ? p.rows.pbeg[1] : p.rows.pbeg[0];
      float2* s0t = s ? s0b : s0a;
      if (slot > G) {
        // Ghat rows: into the owner's registers, and S0 = Ghat[v][r] of every
        // pair of the particle into the spin's table
        if (l < nv) {
          const float2* row = pw + (N + l) * NS;
#pragma unroll
          for (int c = 0; c < kMdRowsMaxN; ++c) {
            const float2 v = c < N ? row[c] : make_float2(0.f, 0.f);
            if (s)
              gh1[c] = v;
            else
              gh0[c] = v;
          }
          for (int k = pb[l]; k < pb[l + 1]; ++k) s0t[k] = row[pl[k] & 255];
        }
      } else {
        // X0^2 (one 16x16 tile, four real products over four k steps) and
        // the pair sums in FP32 (the contraction type); the traces and the
        // determinant algebra in FP64
        {
          typedef Mfma<float> MM;
          const int li = l & 15, lk = l >> 4;
          MM::acc_t rr = MM::zero(), ri = MM::zero(), ir = MM::zero(), ii = MM::zero();
#pragma unroll
          for (int kk = 0; kk < kMdRowsMaxN / 4; ++kk) {
            const int k = 4 * kk + lk;
            const bool ka = li < N && k < N;
            const float2 a = ka ? pw[li * NS + k] : make_float2(0.f, 0.f);
            const float2 b = ka ? pw[k * NS + li] : make_float2(0.f, 0.f);
            rr = MM::mma(a.x, b.x, rr);
            ii = MM::mma(a.y, b.y, ii);
            ri = MM::mma(a.x, b.y, ri);
            ir = MM::mma(a.y, b.x, ir);
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = 4 * lk + v;
            if (row < N && li < N) x2[row * NS + li] = make_float2(rr[v] - ii[v], ri[v] + ir[v]);
          }
        }
        wave_lds_sync();
        double t0r = 0.0, t0i = 0.0, t2r = 0.0, t2i = 0.0;
        if (l < N) {
          const float2 d = pw[l * NS + l], d2 = x2[l * NS + l];
          t0r = d.x;
          t0i = d.y;
          t2r = d2.x;
          t2i = d2.y;
        }
        const Cx trx0 = cx(wave_sum(t0r), wave_sum(t0i)), trx2 = cx(wave_sum(t2r), wave_sum(t2i));
        // the pairs of particle t = l: GX = Ghat[v] X0[:, r], PX = P[v] X0[:, r],
        // GXX = Ghat[v] X0^2[:, r] (sums over the occupied index), and the
        // t^1 / t^2 coefficients of the single excitation r -> v
        const Cx e2 = 0.5 * (trx0 * trx0 - trx2);
        if (l < nv) {
          const float2* pv = pw + (N + l) * NS;
          for (int k = pb[l]; k < pb[l + 1]; ++k) {
            const int r = pl[k] & 255;
            float gxr = 0.f, gxi = 0.f, pxr = 0.f, pxi = 0.f, ggr = 0.f, ggi = 0.f;
#pragma unroll
            for (int c = 0; c < kMdRowsMaxN; ++c) {
              if (c < N) {
                const float2 g = s ? gh1[c] : gh0[c];
                const float2 qv = pv[c], x = pw[c * NS + r], y = x2[c * NS + r];
                gxr = fmaf(g.x, x.x, fmaf(-g.y, x.y, gxr));
                gxi = fmaf(g.x, x.y, fmaf(g.y, x.x, gxi));
                pxr = fmaf(qv.x, x.x, fmaf(-qv.y, x.y, pxr));
                pxi = fmaf(qv.x, x.y, fmaf(qv.y, x.x, pxi));
                ggr = fmaf(g.x, y.x, fmaf(-g.y, y.y, ggr));
                ggi = fmaf(g.x, y.y, fmaf(g.y, y.x, ggi));
              }
            }
            tab[3 * k] = make_float2(gxr, gxi);
            tab[3 * k + 1] = make_float2(pxr, pxi);
            tab[3 * k + 2] = make_float2(ggr, ggi);
            const float2 sv = s0t[k], qv = pv[r], xv = pw[r * NS + r], yv = x2[r * NS + r];
            Cx c1, c2;
            md_single(cx(sv.x, sv.y), cx(qv.x, qv.y), cx(gxr, gxi), cx(pxr, pxi), cx(ggr, ggi),
                      cx(xv.x, xv.y), cx(yv.x, yv.y), trx0, e2, c1, c2);
            e1t[2 * k] = make_double2(c1.r, c1.i);
            e1t[2 * k + 1] = make_double2(c2.r, c2.i);
          }
        }
        wave_lds_sync();
        Cx vn = cx(0, 0);
#pragma unroll
        for (int k = 0; k < DPL; ++k) {
          const unsigned w0 = s ? dxw[k][1][0] : dxw[k][0][0];
          const unsigned w1 = s ? dxw[k][1][1] : dxw[k][0][1];
          const unsigned w2 = s ? dxw[k][1][2] : dxw[k][0][2];
          const int E = (int)(w0 & 3u);
          Cx c1, c2;
          if (E == 0) {
            c1 = trx0;
            c2 = 0.5 * (trx0 * trx0 - trx2);
          } else if (E == 1) {
            const int k1 = (int)(w1 & 0xffffu);
            const double2 a = e1t[2 * k1], b = e1t[2 * k1 + 1];
            c1 = cx(a.x, a.y);
            c2 = cx(b.x, b.y);
          } else {
            md_det_rows<2>(N, NS, w0, w1, w2, pw, x2, tab, s0t, trx0, trx2, c1, c2);
          }
          if (slot < G) {
            if (s == 0) {
              acc[k] = acc[k] + cd[k] * c2;
              c1p[k] = c1;
            } else {
              acc[k] = acc[k] + cu[k] * c2 + coef[k] * (c1p[k] * c1);
              vn = vn + (c1p[k] * cd[k] + cu[k] * c1);
            }
          } else {
            acc[k] = acc[k] + (s ? cu[k] * c1 : cd[k] * c1);
          }
        }
        if (slot < G && s == 1) {
          const double vr = wave_sum(vn.r), vi = wave_sum(vn.i);
          if (l == 0) {
            const Cx v = cdiv(cx(vr, vi), tot);
            if (live) {
              v_re[(long)w * G + slot] = v.r;
              v_im[(long)w * G + slot] = v.i;
            }
            if (!isfinite(v.r) || !isfinite(v.i)) fin = 0;
          }
        }
      }
    }
    __syncthreads();  // step tau done: P(tau) written, P(tau - 1) consumed
    __syncthreads();  // the producers' next operator is in LDS
  }
  double nr = 0.0, ni = 0.0;
#pragma unroll
  for (int k = 0; k < DPL; ++k) {
    nr += acc[k].r;
    ni += acc[k].i;
  }
  nr = wave_sum(nr);
  ni = wave_sum(ni);
  if (l == 0 && live) {
    const Cx e = cdiv(cx(nr, ni), tot);
    eln_re[w] = e.r;
    eln_im[w] = e.i;
    vfin[w] = fin;
  }
}

template <int KS, int DPL>
__global__ __launch_bounds__(512) void k_md_energy_rows(
    MDParams p, MdRowsLds L, int W, const double* __restrict__ thr, const double* __restrict__ thi,
    const double* __restrict__ c0_re, const double* __restrict__ c0_im, const double* tot_re,
    const double* tot_im, double* v_re, double* v_im, double* eln_re, double* eln_im, int* vfin) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int wv = wave_id(), wl = wv >> 1;
  const int w = blockIdx.x * kMdWalkers + wl;
  const bool live = w < W;
  const int wr = live ? w : W - 1;  // the last block's idle walkers read a real one
  // both roles pass the same number of block barriers: 1 + 2 (NPH + 1).
  // Even wavefronts produce, odd ones consume: a block's wavefronts w and
  // w + 4 share a SIMD, so the producers occupy two SIMDs and the consumers
  // (FP64 vector work, which runs slower beside another wavefront's MFMAs)
  // the other two.
  if ((wv & 1) == 0)
    md_rows_producer<KS>(p, L, lds_raw, wl, (long)wr * p.M * p.Nt, thr, thi);
  else
    md_rows_consumer<DPL>(p, L, lds_raw, wl, w, wr, live, c0_re, c0_im, tot_re, tot_im, v_re, v_im,
                          eln_re, eln_im, vfin);
}

// Launches the compact-row kernel when its tables exist and its LDS fits;
// returns false (nothing launched) otherwise.
static bool md_energy_rows(hipStream_t st, int W, const MDParams& p, const double* thr,
                           const double* thi, const double* c0_re, const double* c0_im,
                           const double* tot_re, const double* tot_im, double* v_re, double* v_im,
                           double* eln_re, double* eln_im, int* vfin, size_t max_lds) {
  if (!p.rows.ok || p.M > kMdRowsMaxM || p.n_det > kMdRowsMaxDet || W < 1) return false;
  const int ks = p.rows.KS;
  if (ks != 16 && ks != 32) return false;
  const MdRowsLds L = md_rows_lds(p, ks);
  if ((size_t)L.total > max_lds) return false;
  const int dpl = (p.n_det + 63) / 64;
  const dim3 grid((W + kMdWalkers - 1) / kMdWalkers), block(128 * kMdWalkers);
#define AFQ_MDR_LAUNCH(K, D)                                                                   \
  hipLaunchKernelGGL((k_md_energy_rows<K, D>), grid, block, L.total, st, p, L, W, thr, thi, \
                     c0_re, c0_im, tot_re, tot_im, v_re, v_im, eln_re, eln_im, vfin)
  if (ks == 16) {
    if (dpl <= 1) AFQ_MDR_LAUNCH(16, 1);
    else if (dpl <= 2) AFQ_MDR_LAUNCH(16, 2);
    else AFQ_MDR_LAUNCH(16, 4);
  } else {
    if (dpl <= 1) AFQ_MDR_LAUNCH(32, 1);
    else if (dpl <= 2) AFQ_MDR_LAUNCH(32, 2);
    else AFQ_MDR_LAUNCH(32, 4);
  }
#undef AFQ_MDR_LAUNCH
  return true;
}

// dst (fragment order, see md_rows_tile): slot, J < KS / 4, rt < RP / 16,
// lk < 4, li < 16, jj < 4 -> element (m, c) = (16 J + 4 jj + lk, 16 rt + li)
// = src[slot][m][rowmap[c]] for m < M and c < R, zero otherwise.
__global__ void k_md_rows_gather(int nslot, int M, int KS, int R, int RP,
                                 const int* __restrict__ rowmap, const double* __restrict__ src,
                                 float* __restrict__ dst) {
  const int RTP = RP / 16, KJ = KS / 4;
  const long n = (long)nslot * KJ * RTP * 256;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const int jj = (int)(e & 3), li = (int)((e >> 2) & 15), lk = (int)((e >> 6) & 3);
    const long b = e >> 8;
    const int rt = (int)(b % RTP), J = (int)((b / RTP) % KJ);
    const long slot = b / ((long)RTP * KJ);
    const int m = 16 * J + 4 * jj + lk, c = 16 * rt + li;
    dst[e] = (m < M && c < R) ? (float)src[(slot * M + m) * M + rowmap[c]] : 0.f;
  }
}

hipError_t md_rows_gather(hipStream_t st, int nslot, int M, int KS, int R, int RP,
                          const int* rowmap, const double* src, float* dst) {
  if (nslot < 1 || M < 1 || M > 4 * KS || KS % 4 || RP < 16 || RP % 16 || R > RP)
    return hipErrorInvalidValue;
  const long n = (long)nslot * KS * RP * 4;
  const int blocks = (int)std::min<long>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_md_rows_gather, dim3(blocks), dim3(256), 0, st, nslot, M, KS, R, RP, rowmap,
                     src, dst);
  return hipGetLastError();
}

template <typename T>
hipError_t md_energy(hipStream_t st, int W, const MDParams& p, const double* thr,
                     const double* thi, const double* c0_re, const double* c0_im,
                     const double* tot_re, const double* tot_im, double* v_re, double* v_im,
                     double* eln_re, double* eln_im, int* vfin, size_t max_lds) {
  const int Nmax = p.sp[0].N > p.sp[1].N ? p.sp[0].N : p.sp[1].N;
  const int NPmax = ((Nmax + 15) / 16) * 16;
  size_t lds = (size_t)(2 * 2 * p.MP4 * NPmax + 2 * 2 * p.M * Nmax + 2 * p.M * Nmax) * sizeof(T);
  lds = (lds + 7) & ~(size_t)7;
  lds += (size_t)2 * Nmax * Nmax * sizeof(double) + 16;
  if constexpr (sizeof(T) == 4) {
    if (md_energy_rows(st, W, p, thr, thi, c0_re, c0_im, tot_re, tot_im, v_re, v_im, eln_re, eln_im,
                       vfin, max_lds))
      return hipGetLastError();
  }
  if (lds > max_lds) return hipErrorInvalidValue;
  const int dpt = (p.n_det + 255) / 256;
#define AFQ_MD_LAUNCH(D)                                                                         \
  hipLaunchKernelGGL((k_md_energy<T, D>), dim3(W), dim3(256), lds, st, p, Nmax, NPmax, thr, thi, \
                     c0_re, c0_im, tot_re, tot_im, v_re, v_im, eln_re, eln_im, vfin)
  if (dpt <= 1) AFQ_MD_LAUNCH(1);
  else if (dpt <= 2) AFQ_MD_LAUNCH(2);
  else if (dpt <= 4) AFQ_MD_LAUNCH(4);
  else if (dpt <= 8) AFQ_MD_LAUNCH(8);
  else return hipErrorInvalidValue;
#undef AFQ_MD_LAUNCH
  return hipGetLastError();
}

template hipError_t md_energy<double>(hipStream_t, int, const MDParams&, const double*,
                                      const double*, const double*, const double*, const double*,
                                      const double*, double*, double*, double*, double*, int*,
                                      size_t);
template hipError_t md_energy<float>(hipStream_t, int, const MDParams&, const double*,
                                     const double*, const double*, const double*, const double*,
                                     const double*, double*, double*, double*, double*, int*,
                                     size_t);

}  // namespace afq
