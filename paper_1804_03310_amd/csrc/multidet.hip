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
// and spin (relative to det A), from the reference quantities in LDS.  E (the
// excitation rank, 1 or 2) is a template parameter so that every small E x E
// array lives in registers; holes (h0, h1) and particles (v0, v1).
template <int E, typename T>
__device__ inline void md_det_coeffs_e(int N, int Nmax, int h0, int h1, int v0, int v1,
                                       const T* gr, const T* gi, const T* pr, const T* pi,
                                       const double* x2r, const double* x2i, Cx trx0, Cx trx2,
                                       Cx& c1, Cx& c2) {
  const Cx e2 = 0.5 * (trx0 * trx0 - trx2);
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
