// gfx950 kernels of the phaseless AFQMC walker update (arXiv 1804.03310,
// Sec. II and III).  Wave64, 16x16x4 MFMA tiles for the dense contractions,
// LDS-staged operands, fixed-order reductions (bitwise reproducible).
#include "common.hpp"
#include "kernels.hpp"

namespace afq {

// ===========================================================================
// Real GEMM, 64x64 block tile, 4 waves of 32x32, K staged through LDS in
// chunks of 16.  Used for set-up products (the half rotation, the Q tensor's
// P = R^T R, the multi-determinant operands); the per-step propagator build
// and force bias have their own kernels (qroute.hip).
// ===========================================================================
template <typename TIn, typename TOut, bool A_KMAJ>
__global__ __launch_bounds__(256) void k_gemm_real(int Mr, int Nc, int K, const TIn* __restrict__ A,
                                                   int lda, long sA, const TIn* __restrict__ B, int ldb,
                                                   long sB, TOut* __restrict__ C, int ldc, long sC,
                                                   double alpha) {
  constexpr int BM = 64, BN = 64, KC = 16;
  __shared__ TIn As[KC][BM + 1];
  __shared__ TIn Bs[KC][BN + 1];
  typedef Mfma<TIn> MM;
  const long z = blockIdx.z;
  A += z * sA;
  B += z * sB;
  C += z * sC;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int w = wave_id(), l = lane_id();
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  const int li = l & 15, lk = l >> 4;
  typename MM::acc_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = MM::zero();

  for (int k0 = 0; k0 < K; k0 += KC) {
    for (int e = threadIdx.x; e < KC * BM; e += 256) {
      int kk, mm;
      if (A_KMAJ) { kk = e / BM; mm = e % BM; } else { mm = e / KC; kk = e % KC; }
      const int gm = m0 + mm, gk = k0 + kk;
      TIn v = (TIn)0;
      if (gm < Mr && gk < K) v = A_KMAJ ? A[(long)gk * lda + gm] : A[(long)gm * lda + gk];
      As[kk][mm] = v;
    }
    for (int e = threadIdx.x; e < KC * BN; e += 256) {
      const int kk = e / BN, nn = e % BN;
      const int gk = k0 + kk, gn = n0 + nn;
      Bs[kk][nn] = (gk < K && gn < Nc) ? B[(long)gk * ldb + gn] : (TIn)0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      const TIn a0 = As[kk + lk][wm + li], a1 = As[kk + lk][wm + 16 + li];
      const TIn b0 = Bs[kk + lk][wn + li], b1 = Bs[kk + lk][wn + 16 + li];
      acc[0][0] = MM::mma(a0, b0, acc[0][0]);
      acc[0][1] = MM::mma(a0, b1, acc[0][1]);
      acc[1][0] = MM::mma(a1, b0, acc[1][0]);
      acc[1][1] = MM::mma(a1, b1, acc[1][1]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = m0 + wm + 16 * i + MM::row(lk, v), c = n0 + wn + 16 * j + li;
        if (r < Mr && c < Nc) C[(long)r * ldc + c] = (TOut)(alpha * (double)acc[i][j][v]);
      }
}

template <typename TIn, typename TOut, bool A_KMAJ>
hipError_t gemm_real(hipStream_t st, int Mr, int Nc, int K, const TIn* A, int lda, long sA,
                     const TIn* B, int ldb, long sB, TOut* C, int ldc, long sC, int batch,
                     double alpha) {
  dim3 grid((Nc + 63) / 64, (Mr + 63) / 64, batch);
  hipLaunchKernelGGL((k_gemm_real<TIn, TOut, A_KMAJ>), grid, dim3(256), 0, st, Mr, Nc, K, A, lda,
                     sA, B, ldb, sB, C, ldc, sC, alpha);
  return hipGetLastError();
}

template hipError_t gemm_real<double, double, true>(hipStream_t, int, int, int, const double*, int,
                                                    long, const double*, int, long, double*, int,
                                                    long, int, double);
template hipError_t gemm_real<double, double, false>(hipStream_t, int, int, int, const double*, int,
                                                     long, const double*, int, long, double*, int,
                                                     long, int, double);
// ===========================================================================
// Walker-batched complex GEMM for the one-body factors B1 and the Taylor
// terms of exp(A) (Thouless: the propagator acts on a determinant by a
// matrix product on its orbitals).  Block = one 64x64 output tile of one
// walker, four wavefronts of 32x32 (2x2 MFMA tiles).  The k range goes in
// chunks of 16 through double-buffered LDS: each thread loads its part of the
// next chunk (four consecutive elements of a row, 16-byte or 32-byte reads)
// into registers before the current chunk's MFMAs and stores it after them,
// so one barrier per chunk remains.  A complex product takes three real ones
// (Gauss: P1 = Ar Br, P2 = Ai Bi, P3 = (Ar + Ai)(Br + Bi); re = P1 - P2,
// im = P3 - P1 - P2), a real operator (B1) two.
// ===========================================================================
template <typename T, typename TIn, bool A_CPLX, int MODE>
__global__ __launch_bounds__(256) void k_cgemm_walkers(
    int W, int Mr, int Nc, int K, const T* __restrict__ Ar, const T* __restrict__ Ai, int lda, long sA,
    const TIn* __restrict__ Inr, const TIn* __restrict__ Ini, int ldin, long sIn,
    T* __restrict__ Outr, T* __restrict__ Outi, double* __restrict__ D1r, double* __restrict__ D1i,
    double* __restrict__ D2r, double* __restrict__ D2i, int ldo, long sO, double alpha) {
  constexpr int BM = 64, BN = 64, KC = 16;
  __shared__ T Asr[2][KC][BM + 1];
  __shared__ T Asi[2][A_CPLX ? KC : 1][BM + 1];
  __shared__ T Bsr[2][KC][BN + 1];
  __shared__ T Bsi[2][KC][BN + 1];
  typedef Mfma<T> MM;
  typedef typename MM::acc_t acc_t;
  // Blocks go to the eight XCDs in turn (block b to XCD b mod 8), so the
  // tiles of eight consecutive walkers are interleaved: every tile of walker w
  // lands on XCD w mod 8, whose L2 then serves the A rows and term columns
  // that its tiles share.  Walkers past W (the last group of eight) return.
  const int nmt = (Mr + BM - 1) / BM, ntl = nmt * ((Nc + BN - 1) / BN);
  const long grp = blockIdx.x / (8 * ntl);
  const int rem = (int)(blockIdx.x % (8 * ntl)), tile = rem / 8;
  const long w = grp * 8 + (rem % 8);
  if (w >= W) return;
  const int m0 = (tile % nmt) * BM, n0 = (tile / nmt) * BN;
  if (A_CPLX) { Ar += w * sA; Ai += w * sA; }
  Inr += w * sIn;
  Ini += w * sIn;
  const int wv = wave_id(), l = lane_id();
  const int wm = (wv >> 1) * 32, wn = (wv & 1) * 32;
  const int li = l & 15, lk = l >> 4;
  // staging assignment: A chunk [64 rows][16 k], thread -> row ta, k 4 tq ..;
  // B chunk [16 k][64 columns], thread -> k tb, columns 4 tc ..
  const int ta = threadIdx.x >> 2, tq = (threadIdx.x & 3) * 4;
  const int tb = threadIdx.x >> 4, tc = (threadIdx.x & 15) * 4;
  T pa_r[4], pa_i[4], pb_r[4], pb_i[4];
  auto fetch = [&](int k0) {
    const int gm = m0 + ta, gk = k0 + tq;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const bool ok = gm < Mr && gk + j < K;
      pa_r[j] = ok ? Ar[(long)gm * lda + gk + j] : (T)0;
      pa_i[j] = (A_CPLX && ok) ? Ai[(long)gm * lda + gk + j] : (T)0;
    }
    const int gkb = k0 + tb, gn = n0 + tc;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const bool ok = gkb < K && gn + j < Nc;
      pb_r[j] = ok ? (T)Inr[(long)gkb * ldin + gn + j] : (T)0;
      pb_i[j] = ok ? (T)Ini[(long)gkb * ldin + gn + j] : (T)0;
    }
  };
  auto stage = [&](int buf) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      Asr[buf][tq + j][ta] = pa_r[j];
      if (A_CPLX) Asi[buf][tq + j][ta] = pa_i[j];
      Bsr[buf][tb][tc + j] = pb_r[j];
      Bsi[buf][tb][tc + j] = pb_i[j];
    }
  };
  acc_t p1[2][2], p2[2][2], p3[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) { p1[i][j] = MM::zero(); p2[i][j] = MM::zero(); p3[i][j] = MM::zero(); }
  bool live[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
      live[i][j] = m0 + wm + 16 * i < Mr && n0 + wn + 16 * j < Nc;
  fetch(0);
  stage(0);
  __syncthreads();
  int buf = 0;
  for (int k0 = 0; k0 < K; k0 += KC) {
    const bool more = k0 + KC < K;
    if (more) fetch(k0 + KC);
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      T ar[2], ai[2], br[2], bi[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        ar[i] = Asr[buf][kk + lk][wm + 16 * i + li];
        ai[i] = A_CPLX ? Asi[buf][kk + lk][wm + 16 * i + li] : (T)0;
        br[i] = Bsr[buf][kk + lk][wn + 16 * i + li];
        bi[i] = Bsi[buf][kk + lk][wn + 16 * i + li];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          // 16 x 16 tiles wholly past the last row or column (the remainders of
          // the 64 x 64 block) are not issued
          if (!live[i][j]) continue;
          // real operator: p1 = A Br, p2 = A Bi; complex: Gauss's three
          p1[i][j] = MM::mma(ar[i], br[j], p1[i][j]);
          if (A_CPLX) {
            p2[i][j] = MM::mma(ai[i], bi[j], p2[i][j]);
            p3[i][j] = MM::mma(ar[i] + ai[i], br[j] + bi[j], p3[i][j]);
          } else {
            p2[i][j] = MM::mma(ar[i], bi[j], p2[i][j]);
          }
        }
    }
    if (more) stage(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  const long ob = w * sO;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = m0 + wm + 16 * i + MM::row(lk, v), c = n0 + wn + 16 * j + li;
        if (r >= Mr || c >= Nc) continue;
        const long o = ob + (long)r * ldo + c;
        const double cre = A_CPLX ? (double)p1[i][j][v] - (double)p2[i][j][v] : (double)p1[i][j][v];
        const double cim = A_CPLX ? (double)p3[i][j][v] - (double)p1[i][j][v] - (double)p2[i][j][v]
                                  : (double)p2[i][j][v];
        const double xr = alpha * cre, xi = alpha * cim;
        if (MODE == 0) {
          const double yr = (double)Inr[(long)r * ldin + c] + xr;
          const double yi = (double)Ini[(long)r * ldin + c] + xi;
          D1r[o] = yr;
          D1i[o] = yi;
          if (D2r) { D2r[o] = yr; D2i[o] = yi; }
        } else {
          Outr[o] = (T)xr;
          Outi[o] = (T)xi;
          D1r[o] += xr;
          D1i[o] += xi;
        }
      }
}

template <typename T, typename TIn, bool A_CPLX, int MODE>
hipError_t cgemm_walkers(hipStream_t st, int W, int Mr, int Nc, int K, const T* Ar, const T* Ai,
                         int lda, long sA, const TIn* Inr, const TIn* Ini, int ldin, long sIn,
                         T* Outr, T* Outi, double* D1r, double* D1i, double* D2r, double* D2i,
                         int ldo, long sO, double alpha) {
  const long ntl = (long)((Mr + 63) / 64) * ((Nc + 63) / 64);
  dim3 grid((unsigned)(ntl * 8 * ((W + 7) / 8)));
  hipLaunchKernelGGL((k_cgemm_walkers<T, TIn, A_CPLX, MODE>), grid, dim3(256), 0, st, W, Mr, Nc,
                     K, Ar, Ai, lda, sA, Inr, Ini, ldin, sIn, Outr, Outi, D1r, D1i, D2r, D2i, ldo, sO,
                     alpha);
  return hipGetLastError();
}

#define AFQ_INST_CG(T, TIn, AC, MO)                                                              \
  template hipError_t cgemm_walkers<T, TIn, AC, MO>(                                             \
      hipStream_t, int, int, int, int, const T*, const T*, int, long, const TIn*, const TIn*,    \
      int, long, T*, T*, double*, double*, double*, double*, int, long, double);
AFQ_INST_CG(double, double, false, 0)
AFQ_INST_CG(float, double, false, 0)
AFQ_INST_CG(double, double, true, 1)
AFQ_INST_CG(float, double, true, 1)
AFQ_INST_CG(float, float, true, 1)

// ===========================================================================
// Fields and shifted coefficients (Eq. 2 with the force bias of Sec. II).
// One block per walker.  xbar = -i sqrt(dt)(v - lbar), xs = x - xbar,
// coefficient of L_g in A: i sqrt(dt) xs_g; mean-field log factor
// mf = -i sqrt(dt) sum_g xs_g lbar_g.
// ===========================================================================
template <typename T>
__global__ __launch_bounds__(256) void k_fields_coeff(int W, int G, int ldc, uint64_t seed, uint64_t t,
                                                      int system_id, double dt,
                                                      const double* __restrict__ v_re,
                                                      const double* __restrict__ v_im,
                                                      const double* __restrict__ lbar,
                                                      T* __restrict__ coef, double* mf_re,
                                                      double* mf_im, double* xdump, double* hy_re,
                                                      double* hy_im) {
  __shared__ double red[4];
  const int w = blockIdx.x;
  const double sq = sqrt(dt);
  double sre = 0.0, sim = 0.0, hre = 0.0, him = 0.0;
  const int nq = (G + 3) / 4;
  for (int q = threadIdx.x; q < nq; q += blockDim.x) {
    double z[4];
    gaussian4(seed, t, (uint64_t)w, (uint64_t)q, (uint64_t)system_id, z);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int g = 4 * q + j;
      if (g >= G) break;
      const double x = z[j];
      const double vr = v_re ? v_re[(long)w * G + g] : 0.0;
      const double vi = v_im ? v_im[(long)w * G + g] : 0.0;
      const double lb = lbar ? lbar[g] : 0.0;
      // xbar = -i sq (v - lbar): re = sq*vi, im = -sq*(vr - lb)
      const double xsr = x - sq * vi;        // Re(x - xbar)
      const double xsi = sq * (vr - lb);     // Im(x - xbar)
      // i sq xs = -sq*xsi + i sq*xsr
      if (coef) {
        coef[(long)(2 * w) * ldc + g] = (T)(-sq * xsi);
        coef[(long)(2 * w + 1) * ldc + g] = (T)(sq * xsr);
      }
      // -i sq xs lbar = sq*xsi*lb - i sq*xsr*lb
      sre += sq * xsi * lb;
      sim += -sq * xsr * lb;
      // hybrid importance term x xbar - xbar^2 / 2, xbar = sq vi - i sq (vr - lb)
      const double br = sq * vi, bi = -sq * (vr - lb);
      hre += x * br - 0.5 * (br * br - bi * bi);
      him += x * bi - br * bi;
      if (xdump) xdump[(long)w * G + g] = x;
    }
  }
  if (coef)
    for (int g = G + threadIdx.x; g < ldc; g += blockDim.x) {
      coef[(long)(2 * w) * ldc + g] = (T)0;
      coef[(long)(2 * w + 1) * ldc + g] = (T)0;
    }
  sre = block_sum(sre, red);
  sim = block_sum(sim, red);
  if (threadIdx.x == 0 && mf_re) { mf_re[w] = sre; mf_im[w] = sim; }
  if (hy_re) {
    hre = block_sum(hre, red);
    him = block_sum(him, red);
    if (threadIdx.x == 0) { hy_re[w] = hre; hy_im[w] = him; }
  }
}

template <typename T>
hipError_t fields_coeff(hipStream_t st, int W, int G, int ldc, uint64_t seed, uint64_t t,
                        int system_id, double dt, const double* v_re, const double* v_im,
                        const double* lbar, T* coef, double* mf_re, double* mf_im, double* xdump,
                        double* hy_re, double* hy_im) {
  if (coef && ldc < G) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_fields_coeff<T>), dim3(W), dim3(256), 0, st, W, G, ldc, seed, t, system_id,
                     dt, v_re, v_im, lbar, coef, mf_re, mf_im, xdump, hy_re, hy_im);
  return hipGetLastError();
}
template hipError_t fields_coeff<double>(hipStream_t, int, int, int, uint64_t, uint64_t, int, double,
                                         const double*, const double*, const double*, double*,
                                         double*, double*, double*, double*, double*);
template hipError_t fields_coeff<float>(hipStream_t, int, int, int, uint64_t, uint64_t, int, double,
                                        const double*, const double*, const double*, float*,
                                        double*, double*, double*, double*, double*);

// ===========================================================================
// Overlap, inverse, log det and Theta, FP64 (Sec. II mixed estimates; the
// reference determinant's A and A^-1 of Sec. III).  One block per (walker,
// spin).  The walker's spin block phi and the occupied trial orbitals D_0 are
// staged in LDS when they fit (STAGE), S = D_0^T phi is formed there and
// inverted in place by Gauss-Jordan elimination with row pivoting (the scaled
// pivot row goes to a side buffer so one column costs four barriers), then
// Theta = phi S^-1 and E1 = Tr(htil Theta).
// ===========================================================================
__device__ inline void theta_store(const ThetaOut& to, long w, int M, int Nt, int off, int s, int N,
                                   int m, int b, double vr, double vi) {
  if (to.thr) {
    const long o = (w * M + m) * Nt + off + b;
    to.thr[o] = vr;
    to.thi[o] = vi;
  }
  if (to.sr) {
    const long o = w * to.Ktot + (s ? to.Kp0 : 0) + (long)m * N + b;
    if (to.f32) {
      ((float*)to.sr)[o] = (float)vr;
      ((float*)to.si)[o] = (float)vi;
    } else {
      ((double*)to.sr)[o] = vr;
      ((double*)to.si)[o] = vi;
    }
  }
}

// zeros in the split row's padding of spin s, threads t0, t0 + nt, ...
__device__ inline void theta_pad(const ThetaOut& to, long w, int M, int s, int N, int t0, int nt) {
  if (!to.sr) return;
  const int kp = s ? to.Ktot - to.Kp0 : to.Kp0;
  const long o = w * to.Ktot + (s ? to.Kp0 : 0);
  for (int e = M * N + t0; e < kp; e += nt) {
    if (to.f32) {
      ((float*)to.sr)[o + e] = 0.f;
      ((float*)to.si)[o + e] = 0.f;
    } else {
      ((double*)to.sr)[o + e] = 0.0;
      ((double*)to.si)[o + e] = 0.0;
    }
  }
}

template <bool STAGE>
__global__ __launch_bounds__(512) void k_overlap_theta(int M, int Nt, SpinGeom s0, SpinGeom s1,
                                                       const double* __restrict__ phr,
                                                       const double* __restrict__ phi,
                                                       ThetaOut to, double* ld_re,
                                                       double* ld_im, double* e1_re, double* e1_im) {
  extern __shared__ double lds[];
  __shared__ double red[16];
  __shared__ int piv[AFQ_WAVE];
  __shared__ int pk_sh;
  const int w = blockIdx.x, s = blockIdx.y;
  const SpinGeom g = s ? s1 : s0;
  const int N = g.N, off = g.off;
  const long wb = (long)w * M * Nt;
  if (N == 0) {
    if (threadIdx.x == 0) {
      ld_re[2 * w + s] = 0.0; ld_im[2 * w + s] = 0.0;
      e1_re[2 * w + s] = 0.0; e1_im[2 * w + s] = 0.0;
    }
    return;
  }
  const int ld = N + 1;
  double* Sr = lds;
  double* Si = Sr + N * ld;
  double* fr = Si + N * ld;
  double* fi = fr + N;
  double* rr = fi + N;     // scaled pivot row
  double* ri = rr + N;
  double* Pr = ri + N;     // staged phi block [M][N] (STAGE)
  double* Pi = Pr + (STAGE ? M * N : 0);
  double* Dm = Pi + (STAGE ? M * N : 0);   // staged D_0 [M][N] (STAGE)
  if (STAGE) {
    for (int e = threadIdx.x; e < M * N; e += blockDim.x) {
      const int m = e / N, b = e % N;
      Pr[e] = phr[wb + (long)m * Nt + off + b];
      Pi[e] = phi[wb + (long)m * Nt + off + b];
      Dm[e] = g.C[(long)m * M + b];
    }
    __syncthreads();
  }
  auto PHr = [&](int m, int b) { return STAGE ? Pr[m * N + b] : phr[wb + (long)m * Nt + off + b]; };
  auto PHi = [&](int m, int b) { return STAGE ? Pi[m * N + b] : phi[wb + (long)m * Nt + off + b]; };
  auto D0 = [&](int m, int a) { return STAGE ? Dm[m * N + a] : g.C[(long)m * M + a]; };
  // S[a][b] = sum_m D0[m][a] phi[m][b]
  for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
    const int a = e / N, b = e % N;
    double sr = 0.0, si = 0.0;
    for (int m = 0; m < M; ++m) {
      const double c = D0(m, a);
      sr += c * PHr(m, b);
      si += c * PHi(m, b);
    }
    Sr[a * ld + b] = sr;
    Si[a * ld + b] = si;
  }
  __syncthreads();
  double ldr = 0.0, ldi = 0.0;
  int nswap = 0;
  for (int k = 0; k < N; ++k) {
    if (threadIdx.x < AFQ_WAVE) {
      const int i = k + threadIdx.x;
      double mag = -1.0;
      int idx = i;
      if (i < N) mag = Sr[i * ld + k] * Sr[i * ld + k] + Si[i * ld + k] * Si[i * ld + k];
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) {
        const double om = __shfl_xor(mag, o, AFQ_WAVE);
        const int oi = __shfl_xor(idx, o, AFQ_WAVE);
        if (om > mag || (om == mag && oi < idx)) { mag = om; idx = oi; }
      }
      if (threadIdx.x == 0) { pk_sh = idx; piv[k] = idx; }
    }
    __syncthreads();
    const int p = pk_sh;
    if (p != k) {
      for (int j = threadIdx.x; j < N; j += blockDim.x) {
        double t = Sr[k * ld + j]; Sr[k * ld + j] = Sr[p * ld + j]; Sr[p * ld + j] = t;
        t = Si[k * ld + j]; Si[k * ld + j] = Si[p * ld + j]; Si[p * ld + j] = t;
      }
      ++nswap;
    }
    __syncthreads();
    const zdbl pv = {Sr[k * ld + k], Si[k * ld + k]};
    const zdbl lg = zlog(pv);
    ldr += lg.re;
    ldi += lg.im;
    const zdbl pinv = zdiv(zdbl{1.0, 0.0}, pv);
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
      fr[i] = Sr[i * ld + k];
      fi[i] = Si[i * ld + k];
      const zdbl v = (i == k) ? pinv : zmul(zdbl{Sr[k * ld + i], Si[k * ld + i]}, pinv);
      rr[i] = v.re;
      ri[i] = v.im;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
      const int i = e / N, j = e % N;
      zdbl v;
      if (i == k) {
        v = zdbl{rr[j], ri[j]};
      } else if (j == k) {
        v = zmul(zdbl{-fr[i], -fi[i]}, pinv);
      } else {
        v = zsub(zdbl{Sr[i * ld + j], Si[i * ld + j]}, zmul(zdbl{fr[i], fi[i]}, zdbl{rr[j], ri[j]}));
      }
      Sr[i * ld + j] = v.re;
      Si[i * ld + j] = v.im;
    }
    __syncthreads();
  }
  // undo the row interchanges as column interchanges, last first
  for (int k = N - 1; k >= 0; --k) {
    const int p = piv[k];
    if (p != k) {
      for (int i = threadIdx.x; i < N; i += blockDim.x) {
        double t = Sr[i * ld + k]; Sr[i * ld + k] = Sr[i * ld + p]; Sr[i * ld + p] = t;
        t = Si[i * ld + k]; Si[i * ld + k] = Si[i * ld + p]; Si[i * ld + p] = t;
      }
      __syncthreads();
    }
  }
  // Theta[m][b] = sum_a phi[m][a] Sinv[a][b];  E1 = sum htil[b][m] Theta[m][b]
  double er = 0.0, ei = 0.0;
  for (int e = threadIdx.x; e < M * N; e += blockDim.x) {
    const int m = e / N, b = e % N;
    double tr = 0.0, ti = 0.0;
    for (int a = 0; a < N; ++a) {
      const double pr = PHr(m, a), pi = PHi(m, a);
      const double qr = Sr[a * ld + b], qi = Si[a * ld + b];
      tr += pr * qr - pi * qi;
      ti += pr * qi + pi * qr;
    }
    theta_store(to, w, M, Nt, off, s, N, m, b, tr, ti);
    const double hv = g.htil[(long)b * M + m];
    er += hv * tr;
    ei += hv * ti;
  }
  theta_pad(to, w, M, s, N, threadIdx.x, blockDim.x);
  er = block_sum(er, red);
  ei = block_sum(ei, red);
  if (threadIdx.x == 0) {
    const double pi_ = 3.141592653589793238462643383279;
    ld_re[2 * w + s] = ldr;
    ld_im[2 * w + s] = ldi + ((nswap & 1) ? pi_ : 0.0);
    e1_re[2 * w + s] = er;
    e1_im[2 * w + s] = ei;
  }
}

// Same quantities for N <= 32, one wavefront per (walker, spin) and no block
// barriers.  S = D_0^T phi is an FP64 MFMA product with both operands read
// from global memory in batches of four k steps (the next batch in flight
// while the current one is multiplied).  Each lane then keeps one row half
// (16 complex entries) of S in registers for Gauss-Jordan elimination with
// implicit row pivoting: the pivot row is chosen among the rows not used yet,
// rows never move, and the scaled pivot row is broadcast through LDS.  The
// result R relates to the inverse by S^-1[k][j] = R[pi(k)][pi^-1(j)], pi(k)
// being the pivot row of column k, and is written to LDS in that order;
// det S = sign(pi) prod of the pivots.  Theta = phi S^-1 is a second FP64
// MFMA product over 16-row tiles of phi, three real products per complex one
// (Gauss), with S^-1 held in registers; each tile's operands are requested
// one tile ahead (the first before the elimination starts).
__device__ inline double readlane_d(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <int NT>
struct OvlWave {
  static constexpr int NP = 16 * NT;
  static constexpr int LD = NP + 2;                          // even: 16-byte aligned rows
  // S re/im, two pivot-row buffers (NP re, then NP im), pi
  static constexpr int DOUBLES = 2 * NP * LD + 4 * NP + NP;
};

// The value lane l ^ 32 holds (one cross-half lane swap, no LDS).
__device__ inline double other_half(double v) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)b, hi = (unsigned)(b >> 32);
  const auto rl = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto rh = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  const bool upper = lane_id() >= 32;
  const unsigned nlo = upper ? rl[0] : rl[1], nhi = upper ? rh[0] : rh[1];
  return __longlong_as_double((long long)(((unsigned long long)nhi << 32) | nlo));
}

template <int CTRL>
__device__ inline unsigned long long dpp_u64(unsigned long long x) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)x, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(x >> 32), CTRL, 0xF, 0xF, false);
  return ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
}

// Maximum over each 16-lane row: quad butterflies, then row rotations by 4 and 8.
__device__ inline unsigned long long row_max16_u64(unsigned long long x) {
  unsigned long long y = dpp_u64<0xB1>(x);
  x = y > x ? y : x;
  y = dpp_u64<0x4E>(x);
  x = y > x ? y : x;
  y = dpp_u64<0x124>(x);
  x = y > x ? y : x;
  y = dpp_u64<0x128>(x);
  return y > x ? y : x;
}

__device__ inline unsigned long long readlane_u64(unsigned long long v, int lane) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), lane);
  return ((unsigned long long)hi << 32) | lo;
}

template <int NT>
__global__ __launch_bounds__(128, 2) void k_overlap_theta_wave(int M, int Nt, SpinGeom s0, SpinGeom s1,
                                                            const double* __restrict__ phr,
                                                            const double* __restrict__ phi,
                                                            ThetaOut to, double* ld_re,
                                                            double* ld_im, double* e1_re,
                                                            double* e1_im) {
  typedef OvlWave<NT> L;
  constexpr int NP = L::NP, LD = L::LD, KA = NP / 4;
  using MM = Mfma<double>;
  typedef MM::acc_t acc_t;
  extern __shared__ __attribute__((aligned(16))) double olds[];
  const int wv = wave_id(), l = threadIdx.x & 63;
  const int w = blockIdx.x, s = wv;
  const SpinGeom g = s ? s1 : s0;
  const int N = g.N, off = g.off;
  const long wb = (long)w * M * Nt;
  if (N == 0) {
    if (l == 0) {
      ld_re[2 * w + s] = 0.0; ld_im[2 * w + s] = 0.0;
      e1_re[2 * w + s] = 0.0; e1_im[2 * w + s] = 0.0;
    }
    return;
  }
  double* Sr = olds + wv * L::DOUBLES;
  double* Si = Sr + NP * LD;
  double* prow = Si + NP * LD;  // [2][re, im][NP] pivot-row buffers
  int* piarr = (int*)(Si + NP * LD + 4 * NP);
  const int li = l & 15, lk = l >> 4;
  // ---- S = D_0^T phi (zero padded to NP x NP) ----
  {
    acc_t cr[NT][NT], ci[NT][NT];
#pragma unroll
    for (int I = 0; I < NT; ++I)
#pragma unroll
      for (int J = 0; J < NT; ++J) { cr[I][J] = MM::zero(); ci[I][J] = MM::zero(); }
    const int KS = (M + 3) >> 2;
    double a0[4][NT], r0[4][NT], i0[4][NT], a1[4][NT], r1[4][NT], i1[4][NT];
    auto load = [&](double (&a)[4][NT], double (&br)[4][NT], double (&bi)[4][NT], int kb) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int m = 4 * (kb + j) + lk;
#pragma unroll
        for (int I = 0; I < NT; ++I) {
          const int col = 16 * I + li;
          const bool ok = m < M && col < N;
          a[j][I] = ok ? g.C[(long)m * M + col] : 0.0;
          br[j][I] = ok ? phr[wb + (long)m * Nt + off + col] : 0.0;
          bi[j][I] = ok ? phi[wb + (long)m * Nt + off + col] : 0.0;
        }
      }
    };
    load(a0, r0, i0, 0);
    for (int kb = 0; kb < KS; kb += 4) {
      if (kb + 4 < KS) load(a1, r1, i1, kb + 4);
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int I = 0; I < NT; ++I)
#pragma unroll
          for (int J = 0; J < NT; ++J) {
            cr[I][J] = MM::mma(a0[j][I], r0[j][J], cr[I][J]);
            ci[I][J] = MM::mma(a0[j][I], i0[j][J], ci[I][J]);
          }
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int I = 0; I < NT; ++I) { a0[j][I] = a1[j][I]; r0[j][I] = r1[j][I]; i0[j][I] = i1[j][I]; }
    }
#pragma unroll
    for (int I = 0; I < NT; ++I)
#pragma unroll
      for (int J = 0; J < NT; ++J)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = 16 * I + MM::row(lk, v), c = 16 * J + li;
          Sr[r * LD + c] = cr[I][J][v];
          Si[r * LD + c] = ci[I][J][v];
        }
  }
  wave_lds_sync();
  // first row tile of phi for the Theta product, requested now so that the
  // loads overlap the elimination: A[m = li][a = 4 ka + lk]
  double par[KA], pai[KA];
  auto load_phi_tile = [&](double (&ar)[KA], double (&ai)[KA], int R) {
    const int m = 16 * R + li;
#pragma unroll
    for (int ka = 0; ka < KA; ++ka) {
      const int a = 4 * ka + lk;
      const bool ok = m < M && a < N;
      ar[ka] = ok ? phr[wb + (long)m * Nt + off + a] : 0.0;
      ai[ka] = ok ? phi[wb + (long)m * Nt + off + a] : 0.0;
    }
  };
  load_phi_tile(par, pai, 0);
  // ---- Gauss-Jordan with implicit pivoting, rows in registers ----
  const int i = l & (NP - 1);
  const int h = (NT == 2) ? (l >> 5) : 0;
  const bool owner = (NT == 2) || (l < 16);
  double xr[16], xi[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    xr[c] = Sr[i * LD + 16 * h + c];
    xi[c] = Si[i * LD + 16 * h + c];
  }
  unsigned int used = 0u;
  int mypi = 0, mypinv = 0;
  double pkr = 1.0, pki = 0.0;
  // Pivot steps unrolled in groups of 16 so that the column index within a
  // lane's row half is a constant.  Per step: the column k value of every
  // row (the other half's through a lane swap), the pivot as the largest
  // |S_ik|^2 among unused rows (16-lane DPP maxima, then lanes 0 and 16),
  // the raw pivot row published through LDS, and one update for every row,
  // row_i -= f_i row_p with f_i = S_ik / pv, where the pivot row's own
  // f = 1 - 1 / pv leaves it scaled by 1 / pv; column k becomes 1 / pv in
  // the pivot row and -f_i elsewhere (in-place Gauss-Jordan inverse).
  for (int hk = 0; hk < NT; ++hk) {
#pragma unroll
    for (int ck = 0; ck < 16; ++ck) {
      const int k = 16 * hk + ck;
      if (k >= N) break;
      double fr = xr[ck], fi = xi[ck];
      if (NT == 2) {
        const double orr = other_half(fr), oii = other_half(fi);
        if (h != hk) { fr = orr; fi = oii; }
      }
      // candidate key: |S_ik|^2 (non-negative, so its bits order as unsigned)
      // with the low five mantissa bits replaced by 31 - i (lowest row wins a
      // tie); rows already used and padding rows get 0
      const double mag = fr * fr + fi * fi;
      unsigned long long key =
          (i < N && !((used >> i) & 1u))
              ? (((unsigned long long)__double_as_longlong(mag) & ~31ull) | (unsigned long long)(31 - i))
              : 0ull;
      key = row_max16_u64(key);
      const unsigned long long k0 = readlane_u64(key, 0), k1 = readlane_u64(key, 16);
      const int p = 31 - (int)((k0 > k1 ? k0 : k1) & 31ull);
      used |= 1u << p;
      double* rbr = prow + (k & 1) * 2 * NP;  // re of the row, then im
      double* rbi = rbr + NP;
      if (owner && i == p) {
#pragma unroll
        for (int c = 0; c < 16; c += 2) {
          *(double2*)(rbr + 16 * h + c) = make_double2(xr[c], xr[c + 1]);
          *(double2*)(rbi + 16 * h + c) = make_double2(xi[c], xi[c + 1]);
        }
      }
      const double pvr = readlane_d(fr, p), pvi = readlane_d(fi, p);
      const double rden = 1.0 / (pvr * pvr + pvi * pvi);
      const double pir = pvr * rden, pii = -pvi * rden;
      if (l == k) { pkr = pvr; pki = pvi; mypi = p; }
      if (i == p) mypinv = k;
      double gr, gi;
      if (i == p) {
        gr = 1.0 - pir;
        gi = -pii;
      } else {
        gr = fr * pir - fi * pii;
        gi = fr * pii + fi * pir;
      }
      wave_lds_sync();
#pragma unroll
      for (int c = 0; c < 16; c += 2) {
        const double2 r2 = *(const double2*)(rbr + 16 * h + c);
        const double2 i2 = *(const double2*)(rbi + 16 * h + c);
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const double rr = u ? r2.y : r2.x, ri = u ? i2.y : i2.x;
          // x - g r as two fused multiply-adds per part
          double nr = fma(gi, ri, fma(-gr, rr, xr[c + u]));
          double ni = fma(-gi, rr, fma(-gr, ri, xi[c + u]));
          if (c + u == ck && (NT == 1 || h == hk)) {
            nr = (i == p) ? pir : -gr;
            ni = (i == p) ? pii : -gi;
          }
          xr[c + u] = nr;
          xi[c + u] = ni;
        }
      }
    }
  }
  // ---- log det: pivots and the sign of pi ----
  if (l < N) piarr[l] = mypi;
  wave_lds_sync();
  double lr = 0.0, lim = 0.0, inv = 0.0;
  if (l < N) {
    const zdbl lg = zlog(zdbl{pkr, pki});
    lr = lg.re;
    lim = lg.im;
    const int pk = piarr[l];
    int cnt = 0;
    for (int k2 = l + 1; k2 < N; ++k2) cnt += piarr[k2] < pk;
    inv = (double)cnt;
  }
  lr = wave_sum(lr);
  lim = wave_sum(lim);
  inv = wave_sum(inv);
  // ---- S^-1[pi^-1(i)][pi(j)] = R[i][j] ----
  if (owner && i < N) {
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      const int j = 16 * h + c;
      if (j < N) {
        const int col = piarr[j];
        Sr[mypinv * LD + col] = xr[c];
        Si[mypinv * LD + col] = xi[c];
      }
    }
  }
  wave_lds_sync();
  // ---- Theta = phi S^-1 by 16-row tiles, E1 = Tr(htil Theta) ----
  double sbr[KA][NT], sbi[KA][NT];
#pragma unroll
  for (int ka = 0; ka < KA; ++ka)
#pragma unroll
    for (int J = 0; J < NT; ++J) {
      sbr[ka][J] = Sr[(4 * ka + lk) * LD + 16 * J + li];
      sbi[ka][J] = Si[(4 * ka + lk) * LD + 16 * J + li];
    }
  const int KN = (N + 3) >> 2;
  const int RT = (M + 15) >> 4;
  double er = 0.0, ei = 0.0;
  for (int R = 0; R < RT; ++R) {
    // this tile's h~ entries (clamped to valid entries, used only where
    // stored), and the next tile's phi requested before this tile's MFMAs
    double hvt[NT][4];
#pragma unroll
    for (int J = 0; J < NT; ++J)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = min(16 * R + MM::row(lk, v), M - 1), b = min(16 * J + li, N - 1);
        hvt[J][v] = g.htil[(long)b * M + m];
      }
    if (R > 0) load_phi_tile(par, pai, R);
    // complex product by three real ones (Gauss): p1 = Ar Br, p2 = Ai Bi,
    // p3 = (Ar + Ai)(Br + Bi); re = p1 - p2, im = p3 - p1 - p2
    acc_t p1[NT], p2[NT], p3[NT];
#pragma unroll
    for (int J = 0; J < NT; ++J) { p1[J] = MM::zero(); p2[J] = MM::zero(); p3[J] = MM::zero(); }
#pragma unroll
    for (int ka = 0; ka < KA; ++ka) {
      if (ka < KN) {
        const double as = par[ka] + pai[ka];
#pragma unroll
        for (int J = 0; J < NT; ++J) {
          p1[J] = MM::mma(par[ka], sbr[ka][J], p1[J]);
          p2[J] = MM::mma(pai[ka], sbi[ka][J], p2[J]);
          p3[J] = MM::mma(as, sbr[ka][J] + sbi[ka][J], p3[J]);
        }
      }
    }
#pragma unroll
    for (int J = 0; J < NT; ++J)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = 16 * R + MM::row(lk, v), b = 16 * J + li;
        const double tr = p1[J][v] - p2[J][v], ti = p3[J][v] - p1[J][v] - p2[J][v];
        if (m < M && b < N) {
          theta_store(to, w, M, Nt, off, s, N, m, b, tr, ti);
          er += hvt[J][v] * tr;
          ei += hvt[J][v] * ti;
        }
      }
  }
  theta_pad(to, w, M, s, N, l, AFQ_WAVE);
  er = wave_sum(er);
  ei = wave_sum(ei);
  if (l == 0) {
    const double pi_ = 3.141592653589793238462643383279;
    ld_re[2 * w + s] = lr;
    ld_im[2 * w + s] = lim + ((((int)inv) & 1) ? pi_ : 0.0);
    e1_re[2 * w + s] = er;
    e1_im[2 * w + s] = ei;
  }
}

constexpr int kOvlThreads = 512;  // the block form (N > 32): eight wavefronts
hipError_t overlap_theta(hipStream_t st, int W, int M, int Nt, SpinGeom s0, SpinGeom s1,
                         const double* phr, const double* phi, ThetaOut to, double* ld_re,
                         double* ld_im, double* e1_re, double* e1_im, size_t max_lds) {
  const int N = s0.N > s1.N ? s0.N : s1.N;
  if (N <= 16) {
    const size_t lds = (size_t)2 * OvlWave<1>::DOUBLES * sizeof(double);
    hipLaunchKernelGGL(k_overlap_theta_wave<1>, dim3(W), dim3(128), lds, st, M, Nt, s0, s1, phr,
                       phi, to, ld_re, ld_im, e1_re, e1_im);
    return hipGetLastError();
  }
  if (N <= 32) {
    const size_t lds = (size_t)2 * OvlWave<2>::DOUBLES * sizeof(double);
    hipLaunchKernelGGL(k_overlap_theta_wave<2>, dim3(W), dim3(128), lds, st, M, Nt, s0, s1, phr,
                       phi, to, ld_re, ld_im, e1_re, e1_im);
    return hipGetLastError();
  }
  const size_t base = (size_t)(2 * N * (N + 1) + 4 * N) * sizeof(double);
  const size_t staged = base + (size_t)3 * M * N * sizeof(double);
  if (staged <= 65536 && staged <= max_lds) {
    hipLaunchKernelGGL(k_overlap_theta<true>, dim3(W, 2), dim3(kOvlThreads), staged, st, M, Nt, s0, s1, phr,
                       phi, to, ld_re, ld_im, e1_re, e1_im);
  } else {
    if (base > max_lds) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_overlap_theta<false>, dim3(W, 2), dim3(kOvlThreads), base, st, M, Nt, s0, s1, phr,
                       phi, to, ld_re, ld_im, e1_re, e1_im);
  }
  return hipGetLastError();
}

// ===========================================================================
// Fused exchange / Coulomb / force-bias contraction (Sec. II local energy and
// force bias; the half-rotated form of Eq. Ys).  One block per (walker,
// spin); each wave takes every 4th Cholesky index g and forms
// X_g = Ltil_g Theta (N x N, complex) as 16x16 MFMA tiles, pairing tile
// (I,J) with (J,I) through a per-wave LDS scratch so that Tr(X X) =
// sum_ab X_ab X_ba never leaves the CU.  Theta is staged once in LDS in the
// contraction type T when it fits (THETA_LDS); otherwise the B operand is
// read from the walker's FP64 Theta in global memory (L2 resident).
// ===========================================================================
template <typename T, bool THETA_LDS>
__global__ __launch_bounds__(256) void k_exchange(int M, int MP4, int Nt, int G, SpinGeom s0,
                                                  SpinGeom s1, const double* __restrict__ thr,
                                                  const double* __restrict__ thi,
                                                  double* __restrict__ vs_re,
                                                  double* __restrict__ vs_im, double* exx_re,
                                                  double* exx_im) {
  extern __shared__ unsigned char lds_raw[];
  __shared__ double red[8];
  typedef Mfma<T> MM;
  typedef typename MM::acc_t acc_t;
  const int w = blockIdx.x, s = blockIdx.y;
  const SpinGeom g = s ? s1 : s0;
  const int N = g.N, NP = g.NP, off = g.off;
  const T* __restrict__ Lt = (const T*)g.Lt;
  const int wv = wave_id(), l = lane_id(), li = l & 15, lk = l >> 4;
  if (N == 0) {
    for (int q = threadIdx.x; q < G; q += blockDim.x) {
      vs_re[((long)w * 2 + s) * G + q] = 0.0;
      vs_im[((long)w * 2 + s) * G + q] = 0.0;
    }
    if (threadIdx.x == 0) { exx_re[2 * w + s] = 0.0; exx_im[2 * w + s] = 0.0; }
    return;
  }
  T* Tr = (T*)lds_raw;                       // [MP4][NP] (THETA_LDS)
  T* Ti = Tr + (THETA_LDS ? MP4 * NP : 0);   // [MP4][NP]
  T* scr = Ti + (THETA_LDS ? MP4 * NP : 0);  // 4 waves x 2 x 256
  T* myr = scr + wv * 512;
  T* myi = myr + 256;
  const long wb = (long)w * M * Nt;
  if (THETA_LDS) {
    for (int e = threadIdx.x; e < MP4 * NP; e += blockDim.x) {
      const int m = e / NP, b = e % NP;
      const bool ok = m < M && b < N;
      Tr[e] = ok ? (T)thr[wb + (long)m * Nt + off + b] : (T)0;
      Ti[e] = ok ? (T)thi[wb + (long)m * Nt + off + b] : (T)0;
    }
    __syncthreads();
  }
  // B operand Theta[m][b] (zero outside m < M, b < N)
  auto theta = [&](int m, int b, T& re, T& im) {
    if (THETA_LDS) {
      re = Tr[m * NP + b];
      im = Ti[m * NP + b];
    } else {
      const bool ok = m < M && b < N;
      re = ok ? (T)thr[wb + (long)m * Nt + off + b] : (T)0;
      im = ok ? (T)thi[wb + (long)m * Nt + off + b] : (T)0;
    }
  };
  const int NT = NP / 16;
  double xx_re = 0.0, xx_im = 0.0;
  for (int q = wv; q < G; q += 4) {
    const T* Lq = Lt + (long)q * MP4 * NP;
    double tr_re = 0.0, tr_im = 0.0;
    for (int I = 0; I < NT; ++I) {
      for (int J = I; J < NT; ++J) {
        acc_t pr = MM::zero(), pi = MM::zero(), qr = MM::zero(), qi = MM::zero();
        for (int k = 0; k < MP4; k += 4) {
          const int kr = (k + lk) * NP;
          const T aI = Lq[kr + 16 * I + li];
          T bJr, bJi;
          theta(k + lk, 16 * J + li, bJr, bJi);
          pr = MM::mma(aI, bJr, pr);
          pi = MM::mma(aI, bJi, pi);
          if (I != J) {
            const T aJ = Lq[kr + 16 * J + li];
            T bIr, bIi;
            theta(k + lk, 16 * I + li, bIr, bIi);
            qr = MM::mma(aJ, bIr, qr);
            qi = MM::mma(aJ, bIi, qi);
          }
        }
        // stash the partner tile (J,I) (or (I,I) itself) row-major
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = MM::row(lk, v);
          myr[r * 16 + li] = (I != J) ? qr[v] : pr[v];
          myi[r * 16 + li] = (I != J) ? qi[v] : pi[v];
        }
        wave_lds_sync();
        const double mult = (I != J) ? 2.0 : 1.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = MM::row(lk, v);   // row a within tile (I,J), column b = li
          const double ar = (double)pr[v], ai = (double)pi[v];
          const double br = (double)myr[li * 16 + r], bi = (double)myi[li * 16 + r];
          xx_re += mult * (ar * br - ai * bi);
          xx_im += mult * (ar * bi + ai * br);
          if (I == J && r == li) { tr_re += ar; tr_im += ai; }
        }
        wave_lds_sync();
      }
    }
    tr_re = wave_sum(tr_re);
    tr_im = wave_sum(tr_im);
    if (l == 0) {
      vs_re[((long)w * 2 + s) * G + q] = tr_re;
      vs_im[((long)w * 2 + s) * G + q] = tr_im;
    }
  }
  xx_re = wave_sum(xx_re);
  xx_im = wave_sum(xx_im);
  if (l == 0) { red[wv] = xx_re; red[4 + wv] = xx_im; }
  __syncthreads();
  if (threadIdx.x == 0) {
    exx_re[2 * w + s] = (red[0] + red[1]) + (red[2] + red[3]);
    exx_im[2 * w + s] = (red[4] + red[5]) + (red[6] + red[7]);
  }
}

// Exchange kernel for N <= 16*NT (NT <= 2), one walker and spin per block:
// per Cholesky index all NT x NT tiles of X_g (re and im) are accumulated
// together, so each k step loads NT A values (global, L2 resident) and 2 NT B
// values (LDS) for 2 NT^2 MFMAs; the A operand of the next four k steps (and,
// during the epilogue, of the first four steps of the next g) is prefetched
// into registers.  Theta rows in LDS are unpadded; for 32 columns the two
// 16-column halves of odd rows are swapped so that the lanes reading rows m
// and m+1 hit different banks.  X is stashed row-major once per g in a
// per-wave LDS tile with the same half swap on every other group of four
// rows; the four X_ba values a lane pairs with its four X_ab stay contiguous
// and 16-byte aligned and come back in one 128-bit read.  Per-g partial
// sums are formed in the contraction type and added to FP64 totals.
template <typename T> struct Vec4;
template <> struct Vec4<float> { typedef afq_f4 type; };
template <> struct Vec4<double> { typedef afq_d4 type; };

template <typename T, int NT>
__global__ __launch_bounds__(256, sizeof(T) == 4 ? 4 : 1) void k_exchange_full(int M, int MP4, int Nt, int G, int s_base,
                                                       SpinGeom s0, SpinGeom s1,
                                                       const double* __restrict__ thr,
                                                       const double* __restrict__ thi,
                                                       double* __restrict__ vs_re,
                                                       double* __restrict__ vs_im, double* exx_re,
                                                       double* exx_im) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  __shared__ double red[8];
  typedef Mfma<T> MM;
  typedef typename MM::acc_t acc_t;
  typedef typename Vec4<T>::type v4_t;
  constexpr int NPM = 16 * NT;
  // X stash: the tiles (I, J) with I >= J, row-major; for NT = 2 rows 0-15
  // hold only tile (0, 0) (16 wide), rows 16-31 tiles (1, 0) and (1, 1).
  // Column groups are XOR-swizzled by row group against bank conflicts; a
  // group of four consecutive columns stays contiguous and 16-byte aligned.
  constexpr int XS = NT == 2 ? 768 : 256;  // elements per plane
  auto xaddr = [](int r, int c) {
    if (NT == 1) return r * 16 + c;
    return r < 16 ? r * 16 + (c ^ (((r >> 2) & 3) << 2))
                  : 256 + (r - 16) * 32 + (c ^ (((r >> 2) & 1) << 4));
  };
  const int w = blockIdx.x, s = s_base + blockIdx.y;
  const SpinGeom g = s ? s1 : s0;
  const int N = g.N, off = g.off;
  constexpr int NP = NPM;  // the launch matches NT to this spin's padded width
  const T* __restrict__ Lt = (const T*)g.Lt;
  const int wv = wave_id(), l = lane_id(), li = l & 15, lk = l >> 4;
  if (N == 0) {
    for (int q = threadIdx.x; q < G; q += blockDim.x) {
      vs_re[((long)w * 2 + s) * G + q] = 0.0;
      vs_im[((long)w * 2 + s) * G + q] = 0.0;
    }
    if (threadIdx.x == 0) { exx_re[2 * w + s] = 0.0; exx_im[2 * w + s] = 0.0; }
    return;
  }
  // Theta staged as [m][b mod 16][b / 16][re, im]: the 2 NT B values a lane
  // needs for one k step are contiguous (one 128-bit read for NT = 2)
  T* Bc = (T*)lds_raw;
  T* Xr = Bc + MP4 * 2 * NPM + wv * 2 * XS;
  T* Xi = Xr + XS;
  const long wb = (long)w * M * Nt;
  for (int e = threadIdx.x; e < MP4 * NPM; e += blockDim.x) {
    const int m = e / NPM, b = e % NPM;
    const bool ok = m < M && b < N;
    T* d = Bc + ((m * 16 + (b & 15)) * NT + (b >> 4)) * 2;
    d[0] = ok ? (T)thr[wb + (long)m * Nt + off + b] : (T)0;
    d[1] = ok ? (T)thi[wb + (long)m * Nt + off + b] : (T)0;
  }
  __syncthreads();
  const int KS = MP4 / 4;
  double xx_re = 0.0, xx_im = 0.0;
  T a0[4][NT], a1[4][NT];
  // A operand, four k steps from k step kb of slab q (clamped to the last
  // slab), from the repacked copy: a lane's 4 NT values are contiguous, so
  // they arrive in NT (FP32) or 2 NT (FP64) 128-bit loads
  const int KB = (KS + 3) / 4;
  const T* __restrict__ Apl = (const T*)g.Apk + (long)l * 4 * NT;
  auto load_a = [&](T (&a)[4][NT], int q, int kb) {
    const v4_t* __restrict__ p =
        (const v4_t*)(Apl + ((long)(q < G ? q : G - 1) * KB + kb / 4) * 64 * 4 * NT);
#pragma unroll
    for (int h = 0; h < NT; ++h) {
      const v4_t v = p[h];
#pragma unroll
      for (int e = 0; e < 4; ++e) a[(4 * h + e) / NT][(4 * h + e) % NT] = v[e];
    }
  };
  // this lane's B elements: row 4 k + lk, columns li and 16 + li
  typedef T bvec_t __attribute__((ext_vector_type(2 * NT)));
  const bvec_t* __restrict__ Bl = (const bvec_t*)(Bc + (lk * 16 + li) * 2 * NT);
  load_a(a0, wv, 0);
  for (int q = wv; q < G; q += 4) {
    acc_t cr[NT][NT], ci[NT][NT];
#pragma unroll
    for (int I = 0; I < NT; ++I)
#pragma unroll
      for (int J = 0; J < NT; ++J) { cr[I][J] = MM::zero(); ci[I][J] = MM::zero(); }
    for (int kb = 0; kb < KS; kb += 4) {
      if (kb + 4 < KS) load_a(a1, q, kb + 4);
      else load_a(a1, q + 4, 0);   // first batch of this wave's next g
      // the four k steps' B values are requested together
      bvec_t bq[4];
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (kb + j < KS) bq[j] = Bl[4 * (kb + j) * 16];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (kb + j < KS) {
#pragma unroll
          for (int I = 0; I < NT; ++I)
#pragma unroll
            for (int J = 0; J < NT; ++J) {
              cr[I][J] = MM::mma(a0[j][I], bq[j][2 * J], cr[I][J]);
              ci[I][J] = MM::mma(a0[j][I], bq[j][2 * J + 1], ci[I][J]);
            }
        }
      }
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int I = 0; I < NT; ++I) a0[j][I] = a1[j][I];
    }
    // stash X row-major: lane (li, lk) holds X[16I + row(lk, v)][16J + li].
    // Tr(XX) sums X_ab X_ba over all (a, b); the tile block (I, J), I < J,
    // gives the same sum as (J, I), so only tiles with I >= J are read as
    // partners and only tiles with I <= J are paired (twice for I < J).
#pragma unroll
    for (int I = 0; I < NT; ++I)
#pragma unroll
      for (int J = 0; J < NT; ++J)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          if (I < J) continue;
          const int r = 16 * I + MM::row(lk, v), c = 16 * J + li;
          Xr[xaddr(r, c)] = cr[I][J][v];
          Xi[xaddr(r, c)] = ci[I][J][v];
        }
    wave_lds_sync();
    T pxr = (T)0, pxi = (T)0, ptr = (T)0, pti = (T)0;
#pragma unroll
    for (int I = 0; I < NT; ++I)
#pragma unroll
      for (int J = I; J < NT; ++J) {
        // partners X_ba, b = 16J + li, a = 16I + row(lk, v): for the f32 layout the
        // four a of a lane are consecutive, so one 128-bit read per tile
        T yr[4], yi[4];
        const int rb = 16 * J + li;
        if (MM::row(0, 1) == 1) {
          const int x0 = xaddr(rb, 16 * I + MM::row(lk, 0));
          const v4_t vr = *(const v4_t*)&Xr[x0];
          const v4_t vi = *(const v4_t*)&Xi[x0];
#pragma unroll
          for (int v = 0; v < 4; ++v) { yr[v] = vr[v]; yi[v] = vi[v]; }
        } else {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            yr[v] = Xr[xaddr(rb, 16 * I + MM::row(lk, v))];
            yi[v] = Xi[xaddr(rb, 16 * I + MM::row(lk, v))];
          }
        }
        const T f = (I == J) ? (T)1 : (T)2;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const T xr = f * cr[I][J][v], xi = f * ci[I][J][v];
          pxr += xr * yr[v] - xi * yi[v];
          pxi += xr * yi[v] + xi * yr[v];
          if (MM::row(0, 1) != 1 && I == J && MM::row(lk, v) == li) { ptr += xr; pti += xi; }
        }
      }
    wave_lds_sync();
    xx_re += (double)pxr;
    xx_im += (double)pxi;
    double tr_re, tr_im;
    if (MM::row(0, 1) == 1) {
      // f32 layout: in the lanes that diag16_sum reads, element li & 3 of a
      // diagonal tile is on the diagonal
      const int vd = li & 3;
#pragma unroll
      for (int I = 0; I < NT; ++I) {
        T dr = cr[I][I][0], di = ci[I][I][0];
#pragma unroll
        for (int v = 1; v < 4; ++v) {
          dr = (vd == v) ? cr[I][I][v] : dr;
          di = (vd == v) ? ci[I][I][v] : di;
        }
        ptr += dr;
        pti += di;
      }
      tr_re = (double)diag16_sum((float)ptr);
      tr_im = (double)diag16_sum((float)pti);
    } else {
      tr_re = (double)wave_sum_t(ptr);
      tr_im = (double)wave_sum_t(pti);
    }
    if (l == 0) {
      vs_re[((long)w * 2 + s) * G + q] = tr_re;
      vs_im[((long)w * 2 + s) * G + q] = tr_im;
    }
  }
  xx_re = wave_sum(xx_re);
  xx_im = wave_sum(xx_im);
  if (l == 0) { red[wv] = xx_re; red[4 + wv] = xx_im; }
  __syncthreads();
  if (threadIdx.x == 0) {
    exx_re[2 * w + s] = (red[0] + red[1]) + (red[2] + red[3]);
    exx_im[2 * w + s] = (red[4] + red[5]) + (red[6] + red[7]);
  }
}

// Repack Lt for k_exchange_wide: [g][I][kb][lane][4 k steps], rows past MP4 zero.
template <typename T>
__global__ void k_pack_exchange_a_wide(long n, int MP4, int NP, int KB, const T* __restrict__ Lt,
                                       T* __restrict__ Apk) {
  const int NT = NP / 16;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const int j = (int)(e % 4);
    const int l = (int)((e / 4) % 64);
    const int kb = (int)((e / 256) % KB);
    const int I = (int)((e / (256L * KB)) % NT);
    const long g = e / (256L * KB * NT);
    const int m = 4 * (4 * kb + j) + (l >> 4), a = 16 * I + (l & 15);
    Apk[e] = m < MP4 ? Lt[(g * MP4 + m) * NP + a] : (T)0;
  }
}

template <typename T>
__global__ void k_pack_exchange_a(long n, int MP4, int NP, int KB, const T* __restrict__ Lt,
                                  T* __restrict__ Apk) {
  const int NT = NP / 16;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const int I = (int)(e % NT);
    const int j = (int)((e / NT) % 4);
    const int l = (int)((e / (4 * NT)) % 64);
    const long gkb = e / (4 * NT * 64);
    const int kb = (int)(gkb % KB);
    const long g = gkb / KB;
    const int m = 4 * (4 * kb + j) + (l >> 4), a = 16 * I + (l & 15);
    Apk[e] = m < MP4 ? Lt[(g * MP4 + m) * NP + a] : (T)0;
  }
}

template <typename T>
hipError_t pack_exchange_a(hipStream_t st, int G, int MP4, int NP, const T* Lt, T* Apk) {
  const int KB = (MP4 / 4 + 3) / 4;
  const long n = (long)G * KB * 64 * 4 * (NP / 16);
  if (n == 0) return hipSuccess;
  const int blocks = (int)std::min<long>((n + 255) / 256, 65536);
  if (NP <= 32)
    hipLaunchKernelGGL((k_pack_exchange_a<T>), dim3(blocks), dim3(256), 0, st, n, MP4, NP, KB, Lt, Apk);
  else
    hipLaunchKernelGGL((k_pack_exchange_a_wide<T>), dim3(blocks), dim3(256), 0, st, n, MP4, NP, KB, Lt,
                       Apk);
  return hipGetLastError();
}
template hipError_t pack_exchange_a<double>(hipStream_t, int, int, int, const double*, double*);
template hipError_t pack_exchange_a<float>(hipStream_t, int, int, int, const float*, float*);

// Exchange kernel for 32 < N <= 16 NT (NT = 3, 4), FP32: one walker and spin
// per block of two groups of NT wavefronts; a group takes every other
// Cholesky index and wavefront I of the group computes the row tile I of X_g
// (NT tiles of 16x16, re and im), so its A operand is one value per k step
// (from the repacked copy [g][I][kb][lane][4]) and its B operand the 2 NT
// staged Theta values of the k step.  Tr(XX) pairs the tiles (I, J), J >= I,
// with the stashed tile (J, I) (twice for J > I); each wavefront stashes its
// tiles (I, J), J <= I, and the diagonal trace of tile (I, I) for the group's
// sum.  Two block barriers per pair of Cholesky indices.
template <int NT>
__global__ __launch_bounds__(128 * NT) void k_exchange_wide(int M, int MP4, int Nt, int G,
                                                            int s_base, SpinGeom s0, SpinGeom s1,
                                                            const double* __restrict__ thr,
                                                            const double* __restrict__ thi,
                                                            double* __restrict__ vs_re,
                                                            double* __restrict__ vs_im,
                                                            double* exx_re, double* exx_im) {
  typedef Mfma<float> MM;
  typedef MM::acc_t acc_t;
  constexpr int NPM = 16 * NT, NTRI = NT * (NT + 1) / 2, NW = 2 * NT;
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  __shared__ double red[2 * NW];
  __shared__ float trs[2][2][NT];
  const int w = blockIdx.x, s = s_base + blockIdx.y;
  const SpinGeom g = s ? s1 : s0;
  const int N = g.N, off = g.off;
  const int wv = wave_id(), l = lane_id(), li = l & 15, lk = l >> 4;
  const int grp = wv / NT, I = wv % NT;
  if (N == 0) {
    for (int q = threadIdx.x; q < G; q += blockDim.x) {
      vs_re[((long)w * 2 + s) * G + q] = 0.0;
      vs_im[((long)w * 2 + s) * G + q] = 0.0;
    }
    if (threadIdx.x == 0) { exx_re[2 * w + s] = 0.0; exx_im[2 * w + s] = 0.0; }
    return;
  }
  // Theta as [m][b mod 16][b / 16][re, im]; per group a stash of the NTRI
  // tiles (r, c), r >= c, each 16x16 row-major with column groups swizzled
  float* Bc = (float*)lds_raw;
  float* Xr = Bc + MP4 * 2 * NPM + grp * 2 * NTRI * 256;
  float* Xi = Xr + NTRI * 256;
  const long wb = (long)w * M * Nt;
  for (int e = threadIdx.x; e < MP4 * NPM; e += blockDim.x) {
    const int m = e / NPM, b = e % NPM;
    const bool ok = m < M && b < N;
    float* d = Bc + ((m * 16 + (b & 15)) * NT + (b >> 4)) * 2;
    d[0] = ok ? (float)thr[wb + (long)m * Nt + off + b] : 0.f;
    d[1] = ok ? (float)thi[wb + (long)m * Nt + off + b] : 0.f;
  }
  __syncthreads();
  auto tile = [](int tr, int tc) { return (tr * (tr + 1) / 2 + tc) * 256; };
  auto xsw = [](int r, int c) { return r * 16 + (c ^ (((r >> 2) & 3) << 2)); };
  const int KS = MP4 / 4, KB = (KS + 3) / 4;
  const float* __restrict__ Apl = (const float*)g.Apk + (long)l * 4;
  auto load_a = [&](float (&a)[4], int q, int kb) {
    const afq_f4 v =
        *(const afq_f4*)(Apl + ((((long)(q < G ? q : G - 1) * NT + I) * KB + kb / 4) * 64) * 4);
#pragma unroll
    for (int j = 0; j < 4; ++j) a[j] = v[j];
  };
  const float* __restrict__ Bl = Bc + (lk * 16 + li) * 2 * NT;
  double xx_re = 0.0, xx_im = 0.0;
  float a0[4], a1[4];
  load_a(a0, grp, 0);
  for (int q0 = 0; q0 < G; q0 += 2) {
    const int q = q0 + grp;
    const bool act = q < G;  // uniform over the group; idle groups still meet the barriers
    acc_t cr[NT], ci[NT];
#pragma unroll
    for (int J = 0; J < NT; ++J) { cr[J] = MM::zero(); ci[J] = MM::zero(); }
    if (act) {
      for (int kb = 0; kb < KS; kb += 4) {
        if (kb + 4 < KS) load_a(a1, q, kb + 4);
        else load_a(a1, q + 2, 0);  // first batch of this group's next g
        float bq[4][2 * NT];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if (kb + j < KS) {
            const float* p = Bl + 4 * (kb + j) * 16 * 2 * NT;
#pragma unroll
            for (int h = 0; h < NT / 2; ++h) {
              const afq_f4 v = *(const afq_f4*)(p + 4 * h);
              bq[j][4 * h] = v[0]; bq[j][4 * h + 1] = v[1];
              bq[j][4 * h + 2] = v[2]; bq[j][4 * h + 3] = v[3];
            }
            if (NT & 1) {
              const float2 v = *(const float2*)(p + 2 * NT - 2);
              bq[j][2 * NT - 2] = v.x; bq[j][2 * NT - 1] = v.y;
            }
          }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if (kb + j < KS) {
#pragma unroll
            for (int J = 0; J < NT; ++J) {
              cr[J] = MM::mma(a0[j], bq[j][2 * J], cr[J]);
              ci[J] = MM::mma(a0[j], bq[j][2 * J + 1], ci[J]);
            }
          }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) a0[j] = a1[j];
      }
      // stash tiles (I, J), J <= I: lane (li, lk) holds rows 4 lk + v, column li
#pragma unroll
      for (int J = 0; J < NT; ++J) {
        if (J <= I) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            Xr[tile(I, J) + xsw(4 * lk + v, li)] = cr[J][v];
            Xi[tile(I, J) + xsw(4 * lk + v, li)] = ci[J][v];
          }
        }
      }
      // diagonal of tile (I, I): element li & 3 in the lanes diag16_sum reads
      float dr = 0.f, di = 0.f;
#pragma unroll
      for (int J = 0; J < NT; ++J) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const bool hit = (J == I) && (v == (li & 3));
          dr = hit ? cr[J][v] : dr;
          di = hit ? ci[J][v] : di;
        }
      }
      const float tr = diag16_sum(dr), ti = diag16_sum(di);
      if (l == 0) { trs[grp][0][I] = tr; trs[grp][1][I] = ti; }
    }
    __syncthreads();
    if (act) {
      float pxr = 0.f, pxi = 0.f;
#pragma unroll
      for (int J = 0; J < NT; ++J) {
        if (J >= I) {
          // partner X_ba: row 16 J + li, columns 16 I + 4 lk + v = tile (J, I),
          // local row li, columns 4 lk .. 4 lk + 3
          const int x0 = tile(J, I) + xsw(li, 4 * lk);
          const afq_f4 yr = *(const afq_f4*)&Xr[x0];
          const afq_f4 yi = *(const afq_f4*)&Xi[x0];
          const float f = (J == I) ? 1.f : 2.f;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const float xr = f * cr[J][v], xi = f * ci[J][v];
            pxr += xr * yr[v] - xi * yi[v];
            pxi += xr * yi[v] + xi * yr[v];
          }
        }
      }
      xx_re += (double)pxr;
      xx_im += (double)pxi;
      if (I == 0 && l == 0) {
        double sr = 0.0, si = 0.0;
        for (int t = 0; t < NT; ++t) { sr += (double)trs[grp][0][t]; si += (double)trs[grp][1][t]; }
        vs_re[((long)w * 2 + s) * G + q] = sr;
        vs_im[((long)w * 2 + s) * G + q] = si;
      }
    }
    __syncthreads();
  }
  xx_re = wave_sum(xx_re);
  xx_im = wave_sum(xx_im);
  if (l == 0) { red[wv] = xx_re; red[NW + wv] = xx_im; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sr = 0.0, si = 0.0;
    for (int t = 0; t < NW; ++t) { sr += red[t]; si += red[NW + t]; }
    exx_re[2 * w + s] = sr;
    exx_im[2 * w + s] = si;
  }
}

template <typename T>
hipError_t exchange(hipStream_t st, int W, int M, int MP4, int Nt, int G, SpinGeom s0, SpinGeom s1,
                    const double* thr, const double* thi, double* vs_re, double* vs_im,
                    double* exx_re, double* exx_im, size_t max_lds) {
  const int NP = s0.NP > s1.NP ? s0.NP : s1.NP;
  if (NP <= 32) {
    // one launch per distinct padded width (both spins in one launch when
    // they agree); the kernel's tile count must equal the spin's NP / 16
    // Theta (re, im) [MP4][NPM] plus four waves' X stash (re, im), three
    // 16x16 tiles for NPM = 32 and one for NPM = 16
    auto lds_of = [&](int npm) {
      return (size_t)(2 * MP4 * npm + 4 * 2 * (npm == 32 ? 768 : 256)) * sizeof(T);
    };
    const size_t ld32 = lds_of(32), ld16 = lds_of(16);
    if (ld32 <= max_lds) {
      auto launch = [&](int npm, int s_base, int ny) {
        if (npm == 16)
          hipLaunchKernelGGL((k_exchange_full<T, 1>), dim3(W, ny), dim3(256), ld16, st, M, MP4, Nt,
                             G, s_base, s0, s1, thr, thi, vs_re, vs_im, exx_re, exx_im);
        else
          hipLaunchKernelGGL((k_exchange_full<T, 2>), dim3(W, ny), dim3(256), ld32, st, M, MP4, Nt,
                             G, s_base, s0, s1, thr, thi, vs_re, vs_im, exx_re, exx_im);
      };
      if (s0.NP == s1.NP) {
        launch(s0.NP, 0, 2);
      } else {
        launch(s0.NP, 0, 1);
        launch(s1.NP, 1, 1);
      }
      return hipGetLastError();
    }
  }
  if (sizeof(T) == 4 && NP <= 64 && s0.NP > 32 && s1.NP > 32) {
    // Theta (re, im) [MP4][NP] plus two groups' stashes of NT (NT + 1) / 2 tiles
    auto lds_w = [&](int np) {
      const int nt = np / 16;
      return (size_t)(2 * MP4 * np + 2 * 2 * (nt * (nt + 1) / 2) * 256) * sizeof(float);
    };
    if (lds_w(NP) <= max_lds) {
      auto launch = [&](int np, int s_base, int ny) {
        if (np == 48)
          hipLaunchKernelGGL((k_exchange_wide<3>), dim3(W, ny), dim3(384), lds_w(48), st, M, MP4, Nt,
                             G, s_base, s0, s1, thr, thi, vs_re, vs_im, exx_re, exx_im);
        else
          hipLaunchKernelGGL((k_exchange_wide<4>), dim3(W, ny), dim3(512), lds_w(64), st, M, MP4, Nt,
                             G, s_base, s0, s1, thr, thi, vs_re, vs_im, exx_re, exx_im);
      };
      if (s0.NP == s1.NP) {
        launch(s0.NP, 0, 2);
      } else {
        launch(s0.NP, 0, 1);
        launch(s1.NP, 1, 1);
      }
      return hipGetLastError();
    }
  }
  const size_t lds = (size_t)(2 * MP4 * NP + 4 * 512) * sizeof(T);
  if (lds <= max_lds) {
    hipLaunchKernelGGL((k_exchange<T, true>), dim3(W, 2), dim3(256), lds, st, M, MP4, Nt, G, s0, s1,
                       thr, thi, vs_re, vs_im, exx_re, exx_im);
  } else {
    hipLaunchKernelGGL((k_exchange<T, false>), dim3(W, 2), dim3(256), (size_t)4 * 512 * sizeof(T),
                       st, M, MP4, Nt, G, s0, s1, thr, thi, vs_re, vs_im, exx_re, exx_im);
  }
  return hipGetLastError();
}
template hipError_t exchange<double>(hipStream_t, int, int, int, int, int, SpinGeom, SpinGeom,
                                     const double*, const double*, double*, double*, double*,
                                     double*, size_t);
template hipError_t exchange<float>(hipStream_t, int, int, int, int, int, SpinGeom, SpinGeom,
                                    const double*, const double*, double*, double*, double*,
                                    double*, size_t);

// ===========================================================================
// Per-walker combination (one wave per walker):
// v_g = v_up,g + v_dn,g;  E_L = e_core + E1 + 1/2 sum_g v_g^2 - 1/2 sum_s exx_s.
// ===========================================================================
__global__ __launch_bounds__(256) void k_combine_single(
    int W, int G, double e_core, const double* __restrict__ vs_re, const double* __restrict__ vs_im,
    const double* exx_re, const double* exx_im, const double* e1_re, const double* e1_im,
    const double* ld_re, const double* ld_im, double* __restrict__ v_re, double* __restrict__ v_im,
    double* lsn_re, double* lsn_im, double* eln_re, double* eln_im, int* vfin) {
  const int w = blockIdx.x * 4 + wave_id();
  const int l = lane_id();
  if (w >= W) return;
  double jr = 0.0, ji = 0.0;
  int fin = 1;
  for (int q = l; q < G; q += AFQ_WAVE) {
    const double a = vs_re[((long)w * 2) * G + q] + vs_re[((long)w * 2 + 1) * G + q];
    const double b = vs_im[((long)w * 2) * G + q] + vs_im[((long)w * 2 + 1) * G + q];
    v_re[(long)w * G + q] = a;
    v_im[(long)w * G + q] = b;
    jr += a * a - b * b;
    ji += 2.0 * a * b;
    if (!isfinite(a) || !isfinite(b)) fin = 0;
  }
  jr = wave_sum(jr);
  ji = wave_sum(ji);
  const double f = wave_sum((double)fin);
  if (l == 0) {
    const double er = e_core + (e1_re[2 * w] + e1_re[2 * w + 1]) + 0.5 * jr -
                      0.5 * (exx_re[2 * w] + exx_re[2 * w + 1]);
    const double ei = (e1_im[2 * w] + e1_im[2 * w + 1]) + 0.5 * ji -
                      0.5 * (exx_im[2 * w] + exx_im[2 * w + 1]);
    eln_re[w] = er;
    eln_im[w] = ei;
    lsn_re[w] = ld_re[2 * w] + ld_re[2 * w + 1];
    lsn_im[w] = ld_im[2 * w] + ld_im[2 * w + 1];
    vfin[w] = (f == (double)AFQ_WAVE) ? 1 : 0;
  }
}

hipError_t combine_single(hipStream_t st, int W, int G, double e_core, const double* vs_re,
                          const double* vs_im, const double* exx_re, const double* exx_im,
                          const double* e1_re, const double* e1_im, const double* ld_re,
                          const double* ld_im, double* v_re, double* v_im, double* lsn_re,
                          double* lsn_im, double* eln_re, double* eln_im, int* vfin) {
  hipLaunchKernelGGL(k_combine_single, dim3((W + 3) / 4), dim3(256), 0, st, W, G, e_core, vs_re,
                     vs_im, exx_re, exx_im, e1_re, e1_im, ld_re, ld_im, v_re, v_im, lsn_re, lsn_im,
                     eln_re, eln_im, vfin);
  return hipGetLastError();
}

// ===========================================================================
// Phaseless weight update (Sec. II): log r = log S' - log S + mf,
// W <- W exp(-dt (Re E_L - E_T)) max(0, cos(Im log r)); walkers with a zero
// or non-finite result die.  One thread per walker (SoA, coalesced).
// ===========================================================================
__global__ void k_weight_update(int W, int mode, double dt, double e_trial,
                                const double* __restrict__ lsn_re, const double* __restrict__ lsn_im,
                                const double* __restrict__ eln_re, const double* __restrict__ eln_im,
                                const double* __restrict__ mf_re, const double* __restrict__ mf_im,
                                const int* __restrict__ vfin, double* weight, double* logS_re,
                                double* logS_im, double* eloc_re, double* eloc_im, int* dead,
                                const double* __restrict__ hy_re, const double* __restrict__ hy_im,
                                double e0) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= W) return;
  if (mode == 3 || mode == 4) {
    // hybrid: W |I| exp(-dt (E_0 - E_T)) max(0, cos dtheta), log I = log r + hy;
    // mode 3 also takes the new E_L (a measurement step)
    const double lr = lsn_re[w] - logS_re[w] + mf_re[w];
    const double li = lsn_im[w] - logS_im[w] + mf_im[w];
    const double c = cos(li);
    const double wn = weight[w] * exp(lr + hy_re[w] - dt * (e0 - e_trial)) * (c > 0.0 ? c : 0.0);
    bool ok = isfinite(wn) && isfinite(lr) && isfinite(li) && isfinite(hy_re[w]) &&
              isfinite(hy_im[w]) && isfinite(lsn_re[w]) && isfinite(lsn_im[w]) && vfin[w] &&
              wn > 0.0;
    if (mode == 3) {
      ok = ok && isfinite(eln_re[w]) && isfinite(eln_im[w]);
      eloc_re[w] = eln_re[w];
      eloc_im[w] = eln_im[w];
    }
    weight[w] = ok ? wn : 0.0;
    logS_re[w] = lsn_re[w];
    logS_im[w] = lsn_im[w];
    dead[w] = ok ? 0 : 1;
    return;
  }
  if (mode == 2) {
    logS_re[w] = lsn_re[w];
    logS_im[w] = lsn_im[w];
    return;
  }
  if (mode == 0) {
    logS_re[w] = lsn_re[w];
    logS_im[w] = lsn_im[w];
    eloc_re[w] = eln_re[w];
    eloc_im[w] = eln_im[w];
    return;
  }
  const double lr = lsn_re[w] - logS_re[w] + mf_re[w];
  const double li = lsn_im[w] - logS_im[w] + mf_im[w];
  const double er = eln_re[w], ei = eln_im[w];
  const double c = cos(li);
  const double wn = weight[w] * exp(-dt * (er - e_trial)) * (c > 0.0 ? c : 0.0);
  const bool ok = isfinite(wn) && isfinite(er) && isfinite(ei) && isfinite(lr) && isfinite(li) &&
                  isfinite(lsn_re[w]) && isfinite(lsn_im[w]) && vfin[w] && wn > 0.0;
  weight[w] = ok ? wn : 0.0;
  logS_re[w] = lsn_re[w];
  logS_im[w] = lsn_im[w];
  eloc_re[w] = er;
  eloc_im[w] = ei;
  dead[w] = ok ? 0 : 1;
}

hipError_t weight_update(hipStream_t st, int W, int mode, double dt, double e_trial,
                         const double* lsn_re, const double* lsn_im, const double* eln_re,
                         const double* eln_im, const double* mf_re, const double* mf_im,
                         const int* vfin, double* weight, double* logS_re, double* logS_im,
                         double* eloc_re, double* eloc_im, int* dead, const double* hy_re,
                         const double* hy_im, double e0) {
  hipLaunchKernelGGL(k_weight_update, dim3((W + 255) / 256), dim3(256), 0, st, W, mode, dt,
                     e_trial, lsn_re, lsn_im, eln_re, eln_im, mf_re, mf_im, vfin, weight, logS_re,
                     logS_im, eloc_re, eloc_im, dead, hy_re, hy_im, e0);
  return hipGetLastError();
}

template <typename TP>
__global__ void k_hybrid_finish(int W, int G, int nz, const TP* __restrict__ part_re,
                                const TP* __restrict__ part_im, double* v_re, double* v_im,
                                const double* __restrict__ ld_re, const double* __restrict__ ld_im,
                                double* lsn_re, double* lsn_im, int* vfin) {
  // one block per walker: v_g = sum_z part[z][w][g] (fixed order), flags
  __shared__ int ok_sh;
  const int w = blockIdx.x;
  if (threadIdx.x == 0) ok_sh = 1;
  __syncthreads();
  int ok = 1;
  for (int g = threadIdx.x; g < G; g += blockDim.x) {
    double sr = 0.0, si = 0.0;
    for (int z = 0; z < nz; ++z) {
      sr += (double)part_re[((long)z * W + w) * G + g];
      si += (double)part_im[((long)z * W + w) * G + g];
    }
    v_re[(long)w * G + g] = sr;
    v_im[(long)w * G + g] = si;
    if (!isfinite(sr) || !isfinite(si)) ok = 0;
  }
  if (!ok) ok_sh = 0;
  __syncthreads();
  if (threadIdx.x == 0) {
    lsn_re[w] = ld_re[2 * w] + ld_re[2 * w + 1];
    lsn_im[w] = ld_im[2 * w] + ld_im[2 * w + 1];
    vfin[w] = ok_sh;
  }
}

template <typename TP>
hipError_t hybrid_force_bias_finish(hipStream_t st, int W, int G, int nz, const TP* part_re,
                                    const TP* part_im, double* v_re, double* v_im,
                                    const double* ld_re, const double* ld_im, double* lsn_re,
                                    double* lsn_im, int* vfin) {
  hipLaunchKernelGGL((k_hybrid_finish<TP>), dim3(W), dim3(256), 0, st, W, G, nz, part_re, part_im,
                     v_re, v_im, ld_re, ld_im, lsn_re, lsn_im, vfin);
  return hipGetLastError();
}
template hipError_t hybrid_force_bias_finish<float>(hipStream_t, int, int, int, const float*,
                                                    const float*, double*, double*, const double*,
                                                    const double*, double*, double*, int*);
template hipError_t hybrid_force_bias_finish<double>(hipStream_t, int, int, int, const double*,
                                                     const double*, double*, double*,
                                                     const double*, const double*, double*,
                                                     double*, int*);

__global__ __launch_bounds__(256) void k_reset_dead(int M, int Nt, int G, const int* dead,
                                                    const double* D0, double ref_ls_re,
                                                    double ref_ls_im, double ref_el_re,
                                                    double ref_el_im, const double* vref_re,
                                                    const double* vref_im, double* phr, double* phi,
                                                    double* logS_re, double* logS_im,
                                                    double* eloc_re, double* eloc_im, double* v_re,
                                                    double* v_im) {
  const int w = blockIdx.x;
  if (!dead[w]) return;
  const long n = (long)M * Nt;
  for (long e = threadIdx.x; e < n; e += blockDim.x) {
    phr[(long)w * n + e] = D0[e];
    phi[(long)w * n + e] = 0.0;
  }
  for (int q = threadIdx.x; q < G; q += blockDim.x) {
    v_re[(long)w * G + q] = vref_re[q];
    v_im[(long)w * G + q] = vref_im[q];
  }
  if (threadIdx.x == 0) {
    logS_re[w] = ref_ls_re;
    logS_im[w] = ref_ls_im;
    eloc_re[w] = ref_el_re;
    eloc_im[w] = ref_el_im;
  }
}

hipError_t reset_dead(hipStream_t st, int W, int M, int Nt, int G, const int* dead,
                      const double* D0, double ref_ls_re, double ref_ls_im, double ref_el_re,
                      double ref_el_im, const double* vref_re, const double* vref_im,
                      double* phr, double* phi, double* logS_re, double* logS_im,
                      double* eloc_re, double* eloc_im, double* v_re, double* v_im) {
  hipLaunchKernelGGL(k_reset_dead, dim3(W), dim3(256), 0, st, M, Nt, G, dead, D0, ref_ls_re,
                     ref_ls_im, ref_el_re, ref_el_im, vref_re, vref_im, phr, phi, logS_re, logS_im,
                     eloc_re, eloc_im, v_re, v_im);
  return hipGetLastError();
}

// ===========================================================================
// Mixed energy, one block, fixed-order sums.
// ===========================================================================
__global__ __launch_bounds__(1024) void k_mixed_energy(int W, const double* __restrict__ weight,
                                                       const double* __restrict__ eloc_re,
                                                       double* emix_out, double* den_out) {
  __shared__ double red[16];
  double num = 0.0, den = 0.0;
  for (int w = threadIdx.x; w < W; w += blockDim.x) {
    const double x = weight[w];
    num += x * eloc_re[w];
    den += x;
  }
  num = block_sum(num, red);
  den = block_sum(den, red);
  if (threadIdx.x == 0) {
    if (emix_out) emix_out[0] = num / den;
    if (den_out) den_out[0] = den;
  }
}

hipError_t mixed_energy(hipStream_t st, int W, const double* weight, const double* eloc_re,
                        double* emix_out, double* den_out) {
  hipLaunchKernelGGL(k_mixed_energy, dim3(1), dim3(1024), 0, st, W, weight, eloc_re, emix_out,
                     den_out);
  return hipGetLastError();
}

// ===========================================================================
// Modified Gram-Schmidt per (walker, spin), FP64 (Sec. IV.A: periodic
// orthonormalisation of walker orbitals).  The spin block is staged in LDS
// when it fits in the block's LDS (STAGE; up to 160 KB on gfx950, e.g. 200
// orbitals x 50 electrons) and written back at the end; otherwise it is
// updated in place in global memory.
// ===========================================================================
template <bool STAGE>
__global__ __launch_bounds__(1024) void k_mgs(int M, int Nt, int n_up, int n_dn,
                                              double* __restrict__ phr, double* __restrict__ phi) {
  extern __shared__ double qs[];
  __shared__ double red[16];
  const int w = blockIdx.x, s = blockIdx.y;
  const int N = s ? n_dn : n_up, off = s ? n_up : 0;
  const long wb = (long)w * M * Nt;
  const int wv = wave_id(), l = lane_id(), nw = blockDim.x / AFQ_WAVE;
  double* Qr = qs;
  double* Qi = qs + (STAGE ? M * N : 0);
  if (STAGE) {
    for (int e = threadIdx.x; e < M * N; e += blockDim.x) {
      const int m = e / N, b = e % N;
      Qr[e] = phr[wb + (long)m * Nt + off + b];
      Qi[e] = phi[wb + (long)m * Nt + off + b];
    }
    __syncthreads();
  }
  auto R = [&](int m, int c) -> double& { return STAGE ? Qr[m * N + c] : phr[wb + (long)m * Nt + off + c]; };
  auto I = [&](int m, int c) -> double& { return STAGE ? Qi[m * N + c] : phi[wb + (long)m * Nt + off + c]; };
  for (int j = 0; j < N; ++j) {
    double nrm = 0.0;
    for (int m = threadIdx.x; m < M; m += blockDim.x) {
      const double a = R(m, j), b = I(m, j);
      nrm += a * a + b * b;
    }
    nrm = block_sum(nrm, red);
    const double r = sqrt(nrm);
    for (int m = threadIdx.x; m < M; m += blockDim.x) {
      R(m, j) /= r;
      I(m, j) /= r;
    }
    __syncthreads();
    for (int k = j + 1 + wv; k < N; k += nw) {  // one wavefront per later column
      double dr = 0.0, di = 0.0;
      for (int m = l; m < M; m += AFQ_WAVE) {
        const double qr = R(m, j), qi = I(m, j);
        const double ar = R(m, k), ai = I(m, k);
        dr += qr * ar + qi * ai;   // conj(q) a
        di += qr * ai - qi * ar;
      }
      dr = wave_sum(dr);
      di = wave_sum(di);
      for (int m = l; m < M; m += AFQ_WAVE) {
        const double qr = R(m, j), qi = I(m, j);
        R(m, k) -= dr * qr - di * qi;
        I(m, k) -= dr * qi + di * qr;
      }
    }
    __syncthreads();
  }
  if (STAGE) {
    for (int e = threadIdx.x; e < M * N; e += blockDim.x) {
      const int m = e / N, b = e % N;
      phr[wb + (long)m * Nt + off + b] = Qr[e];
      phi[wb + (long)m * Nt + off + b] = Qi[e];
    }
  }
}

// Same for M <= 64: one wave per (walker, spin), lane m owning row m of every
// column; the columns sit in LDS as [k][m] (each lane touches only its own
// row there), so the only cross-lane step is the sum over rows, a
// fixed-order DPP reduction (16-lane rows, then lanes 0, 16, 32, 48) taken
// for four columns at a time.
template <int CTRL>
__device__ inline double dpp_f64(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

template <int NV>
__device__ inline void wave_sum_dpp(double (&x)[NV]) {
#pragma unroll
  for (int v = 0; v < NV; ++v) x[v] += dpp_f64<0xB1>(x[v]);
#pragma unroll
  for (int v = 0; v < NV; ++v) x[v] += dpp_f64<0x4E>(x[v]);
#pragma unroll
  for (int v = 0; v < NV; ++v) x[v] += dpp_f64<0x124>(x[v]);
#pragma unroll
  for (int v = 0; v < NV; ++v) x[v] += dpp_f64<0x128>(x[v]);
#pragma unroll
  for (int v = 0; v < NV; ++v)
    x[v] = (readlane_d(x[v], 0) + readlane_d(x[v], 16)) + (readlane_d(x[v], 32) + readlane_d(x[v], 48));
}

__global__ __launch_bounds__(128) void k_mgs_wave(int M, int Nt, int n_up, int n_dn,
                                                  double* __restrict__ phr,
                                                  double* __restrict__ phi) {
  extern __shared__ __attribute__((aligned(16))) double mlds[];
  const int w = blockIdx.x, s = wave_id(), l = lane_id();
  const int N = s ? n_dn : n_up, off = s ? n_up : 0;
  const int Nmax = n_up > n_dn ? n_up : n_dn;
  double2* Lc = (double2*)mlds + (long)s * Nmax * M;  // [k][m]
  const long wb = (long)w * M * Nt;
  if (N == 0) return;
  for (int e = l; e < M * N; e += AFQ_WAVE) {
    const int m = e / N, k = e % N;
    Lc[k * M + m] = make_double2(phr[wb + (long)m * Nt + off + k], phi[wb + (long)m * Nt + off + k]);
  }
  wave_lds_sync();
  const bool act = l < M;
  for (int j = 0; j < N; ++j) {
    double2 q = act ? Lc[j * M + l] : make_double2(0.0, 0.0);
    double nv[1] = {q.x * q.x + q.y * q.y};
    wave_sum_dpp<1>(nv);
    const double rinv = 1.0 / sqrt(nv[0]);
    q.x *= rinv;
    q.y *= rinv;
    if (act) Lc[j * M + l] = q;
    for (int k0 = j + 1; k0 < N; k0 += 4) {
      double2 a[4];
      double p[8];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = k0 + u;
        a[u] = (act && k < N) ? Lc[k * M + l] : make_double2(0.0, 0.0);
        p[2 * u] = q.x * a[u].x + q.y * a[u].y;  // conj(q) a
        p[2 * u + 1] = q.x * a[u].y - q.y * a[u].x;
      }
      wave_sum_dpp<8>(p);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = k0 + u;
        if (act && k < N) {
          a[u].x -= p[2 * u] * q.x - p[2 * u + 1] * q.y;
          a[u].y -= p[2 * u] * q.y + p[2 * u + 1] * q.x;
          Lc[k * M + l] = a[u];
        }
      }
    }
  }
  wave_lds_sync();
  for (int e = l; e < M * N; e += AFQ_WAVE) {
    const int m = e / N, k = e % N;
    const double2 v = Lc[k * M + m];
    phr[wb + (long)m * Nt + off + k] = v.x;
    phi[wb + (long)m * Nt + off + k] = v.y;
  }
}

hipError_t mgs(hipStream_t st, int W, int M, int Nt, int n_up, int n_dn, double* phr, double* phi,
               size_t max_lds) {
  const int N = n_up > n_dn ? n_up : n_dn;
  const size_t lds_wave = (size_t)2 * N * M * 2 * sizeof(double);
  if (M <= AFQ_WAVE && lds_wave <= max_lds) {
    hipLaunchKernelGGL(k_mgs_wave, dim3(W), dim3(128), lds_wave, st, M, Nt, n_up, n_dn, phr, phi);
    return hipGetLastError();
  }
  const size_t lds = (size_t)2 * M * N * sizeof(double);
  if (lds <= max_lds)
    hipLaunchKernelGGL(k_mgs<true>, dim3(W, 2), dim3(1024), lds, st, M, Nt, n_up, n_dn, phr, phi);
  else
    hipLaunchKernelGGL(k_mgs<false>, dim3(W, 2), dim3(1024), 0, st, M, Nt, n_up, n_dn, phr, phi);
  return hipGetLastError();
}

// ===========================================================================
// Comb (population control).  The inclusive prefix sums are formed by one
// thread, left to right, so every rounding step is that of a plain loop; each
// tooth z_j = ((j + xi) W_tot) / W then finds the first k with C_k > z_j by a
// binary search over the same prefix array (the result of a left-to-right
// sweep).  The prefix array lives in LDS when W fits, else in global scratch.
// ===========================================================================
__global__ __launch_bounds__(1024) void k_comb_parents(int W, const double* __restrict__ weight,
                                                       uint64_t seed, uint64_t pc_index,
                                                       int system_id, double* __restrict__ cbuf,
                                                       int* parent, double* norm_out, int use_lds) {
  extern __shared__ double cs[];
  __shared__ double sh[2];
  __shared__ int last_sh;
  // LDS: the weights [W], then their prefix sums [W]
  double* C = use_lds ? cs + W : cbuf;
  const double* Wt = use_lds ? cs : weight;
  if (use_lds)
    for (int k = threadIdx.x; k < W; k += blockDim.x) cs[k] = weight[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    // one thread, left to right (the order fixes the rounding of every
    // prefix); the weights are read eight ahead of the sums, from an array
    // the sums are not written to
    double acc = 0.0;
    int last = W - 1;
    int k = 0;
    for (; k + 8 <= W; k += 8) {
      double wk[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) wk[u] = Wt[k + u];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (wk[u] > 0.0) last = k + u;
        acc = acc + wk[u];
        C[k + u] = acc;
      }
    }
    for (; k < W; ++k) {
      const double wk = Wt[k];
      if (wk > 0.0) last = k;
      acc = acc + wk;
      C[k] = acc;
    }
    const PhiloxOut r =
        philox4x64_10(pc_index, 0ull, 0ull, (uint64_t)system_id, seed, AFQ_STREAM_COMB);
    sh[0] = acc;
    sh[1] = u64_to_unit(r.w[0]);
    last_sh = last;
  }
  __syncthreads();
  const double wtot = sh[0], xi = sh[1];
  const int last = last_sh;
  if (!(wtot > 0.0) || !isfinite(wtot)) {
    // every walker dead (or a non-finite weight): the population is left as
    // it is and the norm factor 0 tells the caller
    for (int j = threadIdx.x; j < W; j += blockDim.x) parent[j] = j;
    if (threadIdx.x == 0 && norm_out) norm_out[0] = 0.0;
    return;
  }
  for (int j = threadIdx.x; j < W; j += blockDim.x) {
    const double zj = (((double)j + xi) * wtot) / (double)W;
    int lo = 0, hi = W;  // first index with C[k] > zj in [lo, hi]
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (C[mid] > zj) hi = mid; else lo = mid + 1;
    }
    parent[j] = (lo < W) ? lo : last;
  }
  if (threadIdx.x == 0 && norm_out) norm_out[0] = wtot / (double)W;
}

hipError_t comb_parents(hipStream_t st, int W, const double* weight, uint64_t seed,
                        uint64_t pc_index, int system_id, double* cbuf, int* parent,
                        double* norm_out) {
  const size_t lds = (size_t)2 * W * sizeof(double);
  const int use_lds = lds <= 65536 ? 1 : 0;
  hipLaunchKernelGGL(k_comb_parents, dim3(1), dim3(1024), use_lds ? lds : 0, st, W, weight, seed,
                     pc_index, system_id, cbuf, parent, norm_out, use_lds);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_gather_rows(long row, const int* __restrict__ parent,
                                                     const double* __restrict__ src,
                                                     double* __restrict__ dst) {
  const int j = blockIdx.x;
  const long p = parent[j];
  for (long e = threadIdx.x; e < row; e += blockDim.x) dst[(long)j * row + e] = src[p * row + e];
}

hipError_t gather_rows(hipStream_t st, int W, long row, const int* parent, const double* src,
                       double* dst) {
  hipLaunchKernelGGL(k_gather_rows, dim3(W), dim3(256), 0, st, row, parent, src, dst);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_snap_cols(long row, long c0, int cw,
                                                   const double* __restrict__ src,
                                                   double* __restrict__ snap) {
  const long j = blockIdx.x;
  for (int e = threadIdx.x; e < cw; e += blockDim.x) snap[j * cw + e] = src[j * row + c0 + e];
}

__global__ __launch_bounds__(256) void k_gather_cols(long row, long c0, int cw,
                                                     const int* __restrict__ parent,
                                                     const double* __restrict__ snap,
                                                     double* __restrict__ dst) {
  const long j = blockIdx.x;
  const long p = parent[j];
  for (int e = threadIdx.x; e < cw; e += blockDim.x) dst[j * row + c0 + e] = snap[p * cw + e];
}

hipError_t gather_rows_chunked(hipStream_t st, int W, long row, const int* parent,
                               double* src_dst, double* snap, size_t snap_doubles) {
  if (W < 1 || row < 1) return hipSuccess;
  if (snap_doubles < (size_t)W) return hipErrorInvalidValue;
  const long cw_max = (long)(snap_doubles / (size_t)W);
  for (long c0 = 0; c0 < row; c0 += cw_max) {
    const int cw = (int)std::min(cw_max, row - c0);
    hipLaunchKernelGGL(k_snap_cols, dim3(W), dim3(256), 0, st, row, c0, cw, src_dst, snap);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gather_cols, dim3(W), dim3(256), 0, st, row, c0, cw, parent, snap, src_dst);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Weights after the comb: 1, unless the comb found no positive finite total
// (norm factor 0), in which case they stay as they are.
__global__ void k_comb_weights(int W, const double* __restrict__ norm, double* __restrict__ weight) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < W && norm[0] > 0.0) weight[j] = 1.0;
}

hipError_t comb_weights(hipStream_t st, int W, const double* norm, double* weight) {
  hipLaunchKernelGGL(k_comb_weights, dim3((W + 255) / 256), dim3(256), 0, st, W, norm, weight);
  return hipGetLastError();
}

__global__ void k_fill(double* p, long n, double value) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = value;
}

hipError_t fill(hipStream_t st, double* p, long n, double value) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, value);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_broadcast_rows(long row, const double* __restrict__ src,
                                                        double* __restrict__ dst) {
  const int j = blockIdx.x;
  for (long e = threadIdx.x; e < row; e += blockDim.x) dst[(long)j * row + e] = src[e];
}

hipError_t broadcast_rows(hipStream_t st, int W, long row, const double* src, double* dst) {
  hipLaunchKernelGGL(k_broadcast_rows, dim3(W), dim3(256), 0, st, row, src, dst);
  return hipGetLastError();
}

// lbar_g += sum_{m < M, a < N} Lt[g][m][a] C[m][a]   (one block per g)
__global__ __launch_bounds__(256) void k_lbar(int M, int MP4, int N, int NP,
                                              const double* __restrict__ Lt,
                                              const double* __restrict__ C, double* lbar) {
  __shared__ double red[4];
  const int q = blockIdx.x;
  double s = 0.0;
  for (int e = threadIdx.x; e < M * N; e += blockDim.x) {
    const int m = e / N, a = e % N;
    s += Lt[(long)q * MP4 * NP + (long)m * NP + a] * C[(long)m * M + a];
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) lbar[q] += s;
}

hipError_t lbar_accumulate(hipStream_t st, int G, int M, int MP4, int N, int NP, const double* Lt,
                           const double* C, double* lbar) {
  if (G == 0 || N == 0) return hipSuccess;
  hipLaunchKernelGGL(k_lbar, dim3(G), dim3(256), 0, st, M, MP4, N, NP, Lt, C, lbar);
  return hipGetLastError();
}

__global__ void k_convert(const double* src, float* dst, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (float)src[i];
}

hipError_t convert_f64_f32(hipStream_t st, const double* src, float* dst, long n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_convert, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, dst, n);
  return hipGetLastError();
}

}  // namespace afq

namespace afq {

// ===========================================================================
// Fused one-body propagation for small M (Eq. 3 with Thouless: matrix
// products on the orbitals).  One block per walker:
//   phi1 = phi + (B1 - I) phi,  S = phi1,  T_0 = phi1,
//   T_n = A T_{n-1} / n,  S += T_n  (n = 1..order),  phi = S + (B1 - I) S.
// A and B1 - I (both symmetric) are held in LDS as [i][k] and the current
// term transposed as [c][k], both with k contiguous and row stride LDK (an
// odd multiple of 4), so a lane fetches the four k values of its MFMA steps
// (k = 16 u + 4 lk + j, j = 0..3) with one 16-byte read and eight
// consecutive lanes cover all 32 banks.  The running sum S stays in FP64
// registers of the lanes that own each output element.  Eight waves per
// block.  Terms are rounded to T and the sums accumulate the unrounded FP64
// products, exactly as in the unfused chain.  MT = output tiles per wave;
// SB: every tile of a wave has the same column tile (B fetched once).
// ===========================================================================
constexpr int NWAVE = 8;  // waves per block of the fused propagation

namespace {
// smallest LDK >= MP4 with LDK / 4 odd
inline int taylor_ldk(int MP4) { return ((MP4 / 4) & 1) ? MP4 : MP4 + 4; }
}  // namespace

template <typename T, int MT, bool SB>
__global__ __launch_bounds__(512) void k_propagate_fused(int M, int Nt, int MP4, int LDK, int order,
                                                         int packed, const T* __restrict__ A,
                                                         const T* __restrict__ B1m,
                                                         double* __restrict__ phr,
                                                         double* __restrict__ phi) {
  extern __shared__ __attribute__((aligned(32))) unsigned char lds_raw[];
  typedef Mfma<T> MM;
  typedef typename MM::acc_t acc_t;
  typedef typename Vec4<T>::type t4;
  const int w = blockIdx.x;
  const int wv = wave_id(), l = lane_id(), li = l & 15, lk = l >> 4;
  const long mm = (long)M * M, mn = (long)M * Nt;
  T* Ar = (T*)lds_raw;  // [M][LDK]  A[i][k], zero for k >= M
  T* Ai = Ar + M * LDK;
  T* Bm = Ai + M * LDK;  // (B1 - I)[i][k]
  T* TT = Bm + M * LDK;  // ping-pong term buffers, transposed [Nt][LDK] (re, im)
  auto tt = [&](int buf, int part) { return TT + (2 * buf + part) * Nt * LDK; };
  // phi in the lanes' output ownership: the FP64 running sum S starts from
  // it, and the first term is stored from it (rounded) once A is staged.
  // Requested first, so that these loads overlap the staging of A.
  const long wb = (long)w * mn;
  const int RT = (M + 15) / 16, CT = (Nt + 15) / 16, ntile = RT * CT;
  double sr[MT][4], si[MT][4];
#pragma unroll
  for (int t = 0; t < MT; ++t) {
    const int tile = wv + NWAVE * t;
    const int rt = tile / CT, ct = tile % CT;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * rt + MM::row(lk, v), c = 16 * ct + li;
      const bool ok = tile < ntile && r < M && c < Nt;
      sr[t][v] = ok ? phr[wb + (long)r * Nt + c] : 0.0;
      si[t][v] = ok ? phi[wb + (long)r * Nt + c] : 0.0;
    }
  }
  // Staging of A and B1 - I, rows by wavefronts and the contiguous index by
  // lanes (two passes of 64 cover LDK): each group of RPW rows per wavefront
  // has all its global loads requested before its first LDS store, so that
  // their latencies overlap (a load-store chain per row left most of the
  // block idle during the staging).  Fewer rows per group where registers
  // are scarcer (FP64, one tile per wavefront).
  constexpr int RPW = sizeof(T) == 4 ? (MT >= 2 ? 8 : 4) : 2;
  const long mp = (long)M * (M + 1) / 2;
  const T* Agp = A + (long)w * 2 * mp;
  const T* Agf = A + (long)w * 2 * mm;
  for (int i0 = 0; i0 < MP4; i0 += NWAVE * RPW) {
    T xr[RPW][2], xi[RPW][2], bm[RPW][2];
#pragma unroll
    for (int j = 0; j < RPW; ++j) {
      const int i = i0 + wv + NWAVE * j;  // row of A and B1 - I
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int k = l + AFQ_WAVE * h;  // column of A and B1 - I
        const bool oka = i < M && k < M && (!packed || k >= i);
        const long offp = (long)i * M - (long)i * (i - 1) / 2 - i + k;
        xr[j][h] = oka ? (packed ? Agp[offp] : Agf[(long)i * M + k]) : (T)0;
        xi[j][h] = oka ? (packed ? Agp[mp + offp] : Agf[mm + (long)i * M + k]) : (T)0;
        bm[j][h] = (i < M && k < M) ? B1m[(long)i * M + k] : (T)0;
      }
    }
#pragma unroll
    for (int j = 0; j < RPW; ++j) {
      const int i = i0 + wv + NWAVE * j;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int k = l + AFQ_WAVE * h;
        if (i < M && k < LDK) {
          if (!packed || k >= M) {
            Ar[i * LDK + k] = xr[j][h];  // zero for k >= M
            Ai[i * LDK + k] = xi[j][h];
          } else if (k >= i) {
            // A symmetric, stored as its upper triangle [2][M (M + 1) / 2]
            // (row i holds columns i .. M - 1): entry (i, k) goes to (i, k)
            // and (k, i)
            Ar[i * LDK + k] = xr[j][h];
            Ai[i * LDK + k] = xi[j][h];
            Ar[k * LDK + i] = xr[j][h];
            Ai[k * LDK + i] = xi[j][h];
          }
          Bm[i * LDK + k] = bm[j][h];
        }
      }
    }
  }
  int cur = 0;
  // LDS offsets of the lane's A row and term column per tile, clamped to the
  // last row / column: the clamped lanes read real (finite) entries, so the
  // reads need no mask, and what they give lands only in output rows >= M or
  // columns >= Nt, which are never stored (store_term writes zero rows
  // there).  A wave's tiles beyond the last (tile >= ntile) are computed the
  // same way and never stored, so the products have no branches.
  int arow[MT], bcol[MT];
#pragma unroll
  for (int t = 0; t < MT; ++t) {
    const int tile = wv + NWAVE * t;
    arow[t] = min(16 * (tile / CT) + li, M - 1) * LDK;
    bcol[t] = min(16 * (tile % CT) + li, Nt - 1) * LDK;
  }
  // one product of an M x M operator with the current term: real (B1 - I) or
  // complex A, both from LDS.  The complex product takes three real products
  // (Gauss): P1 = Ar Tr, P2 = Ai Ti, P3 = (Ar + Ai)(Tr + Ti), re = P1 - P2,
  // im = P3 - P1 - P2; the sums Ar + Ai and Tr + Ti are formed from the LDS
  // operands as they are read (on the vector ALU, beside the matrix core).
  auto product = [&](bool cplx, acc_t (&cr)[MT], acc_t (&ci)[MT]) {
    acc_t cs[MT];
#pragma unroll
    for (int t = 0; t < MT; ++t) { cr[t] = MM::zero(); ci[t] = MM::zero(); cs[t] = MM::zero(); }
    const T* br_ = tt(cur, 0);
    const T* bi_ = tt(cur, 1);
    int k0 = 0;
    for (; k0 + 16 <= MP4; k0 += 16) {
      const int kk = k0 + 4 * lk;
      t4 b_r[MT], b_i[MT];
#pragma unroll
      for (int t = 0; t < MT; ++t) {
        if (SB && t > 0) { b_r[t] = b_r[0]; b_i[t] = b_i[0]; continue; }
        b_r[t] = *(const t4*)(br_ + bcol[t] + kk);
        b_i[t] = *(const t4*)(bi_ + bcol[t] + kk);
      }
#pragma unroll
      for (int t = 0; t < MT; ++t) {
        if (cplx) {
          const t4 a_r = *(const t4*)(Ar + arow[t] + kk);
          const t4 a_i = *(const t4*)(Ai + arow[t] + kk);
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            cr[t] = MM::mma(a_r[j], b_r[t][j], cr[t]);
            ci[t] = MM::mma(a_i[j], b_i[t][j], ci[t]);
            cs[t] = MM::mma(a_r[j] + a_i[j], b_r[t][j] + b_i[t][j], cs[t]);
          }
        } else {
          const t4 a = *(const t4*)(Bm + arow[t] + kk);
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            cr[t] = MM::mma(a[j], b_r[t][j], cr[t]);
            ci[t] = MM::mma(a[j], b_i[t][j], ci[t]);
          }
        }
      }
    }
    for (; k0 < MP4; k0 += 4) {  // k tail: one step of four, k = k0 + lk
      const int k = k0 + lk;
#pragma unroll
      for (int t = 0; t < MT; ++t) {
        const T b_r = br_[bcol[t] + k];
        const T b_i = bi_[bcol[t] + k];
        if (cplx) {
          const T a_r = Ar[arow[t] + k];
          const T a_i = Ai[arow[t] + k];
          cr[t] = MM::mma(a_r, b_r, cr[t]);
          ci[t] = MM::mma(a_i, b_i, ci[t]);
          cs[t] = MM::mma(a_r + a_i, b_r + b_i, cs[t]);
        } else {
          const T a = Bm[arow[t] + k];
          cr[t] = MM::mma(a, b_r, cr[t]);
          ci[t] = MM::mma(a, b_i, ci[t]);
        }
      }
    }
    if (cplx) {  // cr = P1, ci = P2, cs = P3
#pragma unroll
      for (int t = 0; t < MT; ++t) {
        const acc_t p1 = cr[t], p2 = ci[t];
        cr[t] = p1 - p2;
        ci[t] = cs[t] - p1 - p2;
      }
    }
  };
  // term^T[c][r] for the lane's rows; rows M .. MP4 - 1 receive zeros (the k
  // padding of the next product), rows from MP4 on are not stored
  auto store_term = [&](int buf, const double (&xr)[MT][4], const double (&xi)[MT][4]) {
    T* outr = tt(buf, 0);
    T* outi = tt(buf, 1);
#pragma unroll
    for (int t = 0; t < MT; ++t) {
      const int tile = wv + NWAVE * t;
      const int rt = tile / CT, ct = tile % CT, c = 16 * ct + li;
      if (tile >= ntile || c >= Nt) continue;
      if (sizeof(T) == 4) {
        const int r0 = 16 * rt + 4 * lk;  // rows r0 .. r0 + 3 (MP4 is a multiple of 4)
        if (r0 < MP4) {
          t4 vr, vi;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            vr[v] = r0 + v < M ? (T)xr[t][v] : (T)0;
            vi[v] = r0 + v < M ? (T)xi[t][v] : (T)0;
          }
          *(t4*)(outr + c * LDK + r0) = vr;
          *(t4*)(outi + c * LDK + r0) = vi;
        }
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = 16 * rt + MM::row(lk, v);
          if (r < MP4) {
            outr[c * LDK + r] = r < M ? (T)xr[t][v] : (T)0;
            outi[c * LDK + r] = r < M ? (T)xi[t][v] : (T)0;
          }
        }
      }
    }
  };
  // the first term: phi, stored transposed from the lanes' S (rows M .. MP4
  // - 1 zero); the block's barrier also publishes A and B1 - I
  store_term(cur, sr, si);
  __syncthreads();
  acc_t cr[MT], ci[MT];
  double xr[MT][4], xi[MT][4];
  // phi1 = phi + (B1 - I) phi
  product(false, cr, ci);
#pragma unroll
  for (int t = 0; t < MT; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      sr[t][v] += (double)cr[t][v];
      si[t][v] += (double)ci[t][v];
    }
  store_term(cur ^ 1, sr, si);
  __syncthreads();
  cur ^= 1;
  // Taylor terms
  for (int n = 1; n <= order; ++n) {
    const double alpha = 1.0 / n;
    product(true, cr, ci);
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        xr[t][v] = alpha * (double)cr[t][v];
        xi[t][v] = alpha * (double)ci[t][v];
        sr[t][v] += xr[t][v];
        si[t][v] += xi[t][v];
      }
    if (n < order) {
      store_term(cur ^ 1, xr, xi);
      __syncthreads();
      cur ^= 1;
    }
  }
  // phi = S + (B1 - I) S
  store_term(cur ^ 1, sr, si);
  __syncthreads();
  cur ^= 1;
  product(false, cr, ci);
#pragma unroll
  for (int t = 0; t < MT; ++t) {
    const int tile = wv + NWAVE * t;
    const int rt = tile / CT, ct = tile % CT;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * rt + MM::row(lk, v), c = 16 * ct + li;
      if (tile < ntile && r < M && c < Nt) {
        phr[wb + (long)r * Nt + c] = sr[t][v] + (double)cr[t][v];
        phi[wb + (long)r * Nt + c] = si[t][v] + (double)ci[t][v];
      }
    }
  }
}

namespace {
size_t taylor_lds(int M, int Nt, size_t elem) {
  const int MP4 = ((M + 3) / 4) * 4;
  return (size_t)(3 * M + 4 * Nt) * taylor_ldk(MP4) * elem;
}
}  // namespace

template <typename T>
hipError_t propagate_fused(hipStream_t st, int W, int M, int Nt, int order, bool packed,
                           const T* A, const T* B1m, double* phr, double* phi, size_t max_lds) {
  const int MP4 = ((M + 3) / 4) * 4, LDK = taylor_ldk(MP4);
  const int CT = (Nt + 15) / 16;
  const int ntile = ((M + 15) / 16) * CT;
  const size_t lds = taylor_lds(M, Nt, sizeof(T));
  if (lds > max_lds || ntile > 8 * NWAVE) return hipErrorInvalidValue;
  const int mt = (ntile + NWAVE - 1) / NWAVE;
  const bool sb = NWAVE % CT == 0;
#define AFQ_PF(MTV, SBV)                                                                          \
  hipLaunchKernelGGL((k_propagate_fused<T, MTV, SBV>), dim3(W), dim3(64 * NWAVE), lds, st, M, Nt,   \
                     MP4, LDK, order, packed ? 1 : 0, A, B1m, phr, phi)
  if (mt <= 1) AFQ_PF(1, false);
  else if (mt <= 2) { if (sb) AFQ_PF(2, true); else AFQ_PF(2, false); }
  else if (mt <= 4) { if (sb) AFQ_PF(4, true); else AFQ_PF(4, false); }
  else AFQ_PF(8, false);
#undef AFQ_PF
  return hipGetLastError();
}

bool propagate_fused_fits(int M, int Nt, size_t elem, size_t max_lds) {
  const int ntile = ((M + 15) / 16) * ((Nt + 15) / 16);
  return taylor_lds(M, Nt, elem) <= max_lds && ntile <= 8 * NWAVE;
}

template hipError_t propagate_fused<float>(hipStream_t, int, int, int, int, bool, const float*,
                                           const float*, double*, double*, size_t);
template hipError_t propagate_fused<double>(hipStream_t, int, int, int, int, bool, const double*,
                                            const double*, double*, double*, size_t);

}  // namespace afq
