// BF16 contractions (BF16 inputs, FP32 accumulation) for the propagator build
// sum_g c_{w,g} L_g and the fused exchange / force-bias contraction
// X_g = Ltil_g Theta (Sec. II; Sec. III single precision).  Operands are laid
// out with the contraction index contiguous so that one 16-byte load gives a
// lane its eight k values.
#include "common.hpp"
#include "kernels.hpp"

namespace afq {

__global__ void k_convert_bf16(const double* src, __bf16* dst, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (__bf16)(float)src[i];
}

hipError_t convert_f64_bf16(hipStream_t st, const double* src, void* dst, long n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_convert_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src,
                     (__bf16*)dst, n);
  return hipGetLastError();
}

// The second term of the split x = hi + lo in bf16: lo = bf16(x - hi),
// hi = bf16(x) (so hi + lo carries about 16 significant bits).
__device__ inline __bf16 bf16_lo(double x) {
  const __bf16 hi = (__bf16)(float)x;
  return (__bf16)(float)(x - (double)(float)hi);
}

__global__ void k_convert_bf16_lo(const double* src, __bf16* dst, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = bf16_lo(src[i]);
}

hipError_t convert_f64_bf16_lo(hipStream_t st, const double* src, void* dst, long n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_convert_bf16_lo, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src,
                     (__bf16*)dst, n);
  return hipGetLastError();
}

// Fragment order of an operand with 16 NT rows and 32 KC columns as one
// 16x16x32 bf16 MFMA reads it: [I][kc][lane] groups of eight, lane = li + 16 lk
// holding row 16 I + li, columns 32 kc + 8 lk .. 32 kc + 8 lk + 7.
//
// Ltil_g (rows a < NP, columns m < MP4 read from the FP64 [G][MP4][NP] copy)
// into that order, one fragment per thread; lo (nullable) receives the
// split's second terms.
__global__ void k_pack_ltilde_bf16(long nfrag, int MP4, int NP, int NTX, int KC,
                                   const double* __restrict__ src, afq_bf8* __restrict__ hi,
                                   afq_bf8* __restrict__ lo) {
  const long f = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nfrag) return;
  const int lane = (int)(f & 63);
  long r = f >> 6;
  const int kc = (int)(r % KC);
  r /= KC;
  const int I = (int)(r % NTX);
  const long g = r / NTX;
  const int a = 16 * I + (lane & 15), m0 = 32 * kc + 8 * (lane >> 4);
  afq_bf8 h, o;
  for (int e = 0; e < 8; ++e) {
    const int m = m0 + e;
    const double x = (m < MP4 && a < NP) ? src[(g * MP4 + m) * NP + a] : 0.0;
    h[e] = (__bf16)(float)x;
    o[e] = bf16_lo(x);
  }
  hi[f] = h;
  if (lo) lo[f] = o;
}

hipError_t pack_ltilde_bf16(hipStream_t st, int G, int MP4, int NP, int NPX, int MP32,
                            const double* src, void* hi, void* lo) {
  const long nfrag = (long)G * (NPX / 16) * (MP32 / 32) * 64;
  if (nfrag <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pack_ltilde_bf16, dim3((unsigned)((nfrag + 255) / 256)), dim3(256), 0, st,
                     nfrag, MP4, NP, NPX / 16, MP32 / 32, src, (afq_bf8*)hi, (afq_bf8*)lo);
  return hipGetLastError();
}

// C[m][n] = alpha * sum_k A[m][k] B[k][n], A row-major [Mr][lda] bf16 (k contiguous),
// B row-major [K][ldb] bf16; 64x64 block tile, K chunks of 32 staged in LDS with
// k contiguous for both operands.  X3: the operands are split in two bf16
// terms (A = A + Al, B = B + Bl) and C takes the three products
// A B + A Bl + Al B (the Al Bl term, of relative size 2^-18, is dropped),
// all accumulated in FP32.
template <typename TOut, bool X3>
__global__ __launch_bounds__(256) void k_gemm_bf16(int Mr, int Nc, int K, const __bf16* __restrict__ A,
                                                   const __bf16* __restrict__ Al, int lda,
                                                   const __bf16* __restrict__ B,
                                                   const __bf16* __restrict__ Bl, int ldb,
                                                   TOut* __restrict__ C, int ldc, double alpha) {
  constexpr int BM = 64, BN = 64, KC = 32, LDK = KC + 8, NS = X3 ? 2 : 1;
  __shared__ __attribute__((aligned(16))) __bf16 As[NS][BM][LDK];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[NS][BN][LDK];
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int w = wave_id(), l = lane_id();
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  const int li = l & 15, lk = l >> 4;
  afq_f4 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = afq_f4{0.f, 0.f, 0.f, 0.f};
  const __bf16 zero = (__bf16)0.0f;
  for (int k0 = 0; k0 < K; k0 += KC) {
    for (int e = threadIdx.x; e < BM * KC; e += 256) {
      const int mm = e / KC, kk = e % KC;
      const int gm = m0 + mm, gk = k0 + kk;
      const bool ok = gm < Mr && gk < K;
      As[0][mm][kk] = ok ? A[(long)gm * lda + gk] : zero;
      if (X3) As[NS - 1][mm][kk] = ok ? Al[(long)gm * lda + gk] : zero;
    }
    for (int e = threadIdx.x; e < BN * KC; e += 256) {
      const int kk = e / BN, nn = e % BN;
      const int gk = k0 + kk, gn = n0 + nn;
      const bool ok = gk < K && gn < Nc;
      Bs[0][nn][kk] = ok ? B[(long)gk * ldb + gn] : zero;
      if (X3) Bs[NS - 1][nn][kk] = ok ? Bl[(long)gk * ldb + gn] : zero;
    }
    __syncthreads();
    afq_bf8 a[2], b[2];
    for (int i = 0; i < 2; ++i) {
      a[i] = *(const afq_bf8*)&As[0][wm + 16 * i + li][8 * lk];
      b[i] = *(const afq_bf8*)&Bs[0][wn + 16 * i + li][8 * lk];
    }
    if (X3) {
      afq_bf8 al[2], bl[2];
      for (int i = 0; i < 2; ++i) {
        al[i] = *(const afq_bf8*)&As[NS - 1][wm + 16 * i + li][8 * lk];
        bl[i] = *(const afq_bf8*)&Bs[NS - 1][wn + 16 * i + li][8 * lk];
      }
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
          acc[i][j] = mfma_bf16(al[i], b[j], acc[i][j]);
          acc[i][j] = mfma_bf16(a[i], bl[j], acc[i][j]);
        }
    }
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) acc[i][j] = mfma_bf16(a[i], b[j], acc[i][j]);
    __syncthreads();
  }
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int v = 0; v < 4; ++v) {
        const int r = m0 + wm + 16 * i + row_bf16(lk, v), c = n0 + wn + 16 * j + li;
        if (r < Mr && c < Nc) C[(long)r * ldc + c] = (TOut)(alpha * (double)acc[i][j][v]);
      }
}

template <typename TOut>
hipError_t gemm_bf16(hipStream_t st, int Mr, int Nc, int K, const void* A, const void* Al, int lda,
                     const void* B, const void* Bl, int ldb, TOut* C, int ldc, double alpha) {
  dim3 grid((Nc + 63) / 64, (Mr + 63) / 64);
  if (Al && Bl)
    hipLaunchKernelGGL((k_gemm_bf16<TOut, true>), grid, dim3(256), 0, st, Mr, Nc, K,
                       (const __bf16*)A, (const __bf16*)Al, lda, (const __bf16*)B,
                       (const __bf16*)Bl, ldb, C, ldc, alpha);
  else
    hipLaunchKernelGGL((k_gemm_bf16<TOut, false>), grid, dim3(256), 0, st, Mr, Nc, K,
                       (const __bf16*)A, nullptr, lda, (const __bf16*)B, nullptr, ldb, C, ldc,
                       alpha);
  return hipGetLastError();
}
template hipError_t gemm_bf16<float>(hipStream_t, int, int, int, const void*, const void*, int,
                                     const void*, const void*, int, float*, int, double);
template hipError_t gemm_bf16<double>(hipStream_t, int, int, int, const void*, const void*, int,
                                      const void*, const void*, int, double*, int, double);

// Fields and shifted coefficients written as coef[2w + part][g] in bf16 (the
// contraction index g contiguous).  Same arithmetic as fields_coeff.
__global__ __launch_bounds__(256) void k_fields_coeff_bf16(int W, int G, int ldg, uint64_t seed,
                                                           uint64_t t, int system_id, double dt,
                                                           const double* __restrict__ v_re,
                                                           const double* __restrict__ v_im,
                                                           const double* __restrict__ lbar,
                                                           __bf16* __restrict__ coef,
                                                           __bf16* __restrict__ coef_lo,
                                                           double* mf_re, double* mf_im,
                                                           double* hy_re, double* hy_im) {
  __shared__ double red[4];
  const int w = blockIdx.x;
  const double sq = sqrt(dt);
  double sre = 0.0, sim = 0.0, hre = 0.0, him = 0.0;
  const int nq = (G + 3) / 4;
  for (int q = threadIdx.x; q < nq; q += blockDim.x) {
    double z[4];
    gaussian4(seed, t, (uint64_t)w, (uint64_t)q, (uint64_t)system_id, z);
    for (int j = 0; j < 4; ++j) {
      const int g = 4 * q + j;
      if (g >= G) break;
      const double vr = v_re[(long)w * G + g], vi = v_im[(long)w * G + g], lb = lbar[g];
      const double xsr = z[j] - sq * vi;
      const double xsi = sq * (vr - lb);
      coef[(long)(2 * w) * ldg + g] = (__bf16)(float)(-sq * xsi);
      coef[(long)(2 * w + 1) * ldg + g] = (__bf16)(float)(sq * xsr);
      if (coef_lo) {
        coef_lo[(long)(2 * w) * ldg + g] = bf16_lo(-sq * xsi);
        coef_lo[(long)(2 * w + 1) * ldg + g] = bf16_lo(sq * xsr);
      }
      sre += sq * xsi * lb;
      sim += -sq * xsr * lb;
      const double br = sq * vi, bi = -sq * (vr - lb);
      hre += z[j] * br - 0.5 * (br * br - bi * bi);
      him += z[j] * bi - br * bi;
    }
  }
  sre = block_sum(sre, red);
  sim = block_sum(sim, red);
  if (threadIdx.x == 0) { mf_re[w] = sre; mf_im[w] = sim; }
  if (hy_re) {
    hre = block_sum(hre, red);
    him = block_sum(him, red);
    if (threadIdx.x == 0) { hy_re[w] = hre; hy_im[w] = him; }
  }
}

hipError_t fields_coeff_bf16(hipStream_t st, int W, int G, int ldg, uint64_t seed, uint64_t t,
                             int system_id, double dt, const double* v_re, const double* v_im,
                             const double* lbar, void* coef, void* coef_lo, double* mf_re,
                             double* mf_im, double* hy_re, double* hy_im) {
  hipLaunchKernelGGL(k_fields_coeff_bf16, dim3(W), dim3(256), 0, st, W, G, ldg, seed, t, system_id,
                     dt, v_re, v_im, lbar, (__bf16*)coef, (__bf16*)coef_lo, mf_re, mf_im, hy_re,
                     hy_im);
  return hipGetLastError();
}

// Index of the tile pair (I, J), I <= J, among the NT (NT + 1) / 2: the
// diagonal pairs first, then I < J in row order.
__host__ __device__ constexpr int xch_pair(int NT, int I, int J) {
  return I == J ? I : NT + I * (2 * NT - I - 1) / 2 + (J - I - 1);
}

// One wavefront's share of the fused exchange: every fourth g from wq on and,
// for each, the tile pairs LO <= xch_pair < HI (role 0 of NR = 2, or all of
// them for NR = 1, holds the diagonal pairs and so the traces).  Over the k
// chunks it accumulates X_IJ = Ltil_I Theta_J and, for I < J, the tile of X^T
// at the same place, X^T_IJ = Theta_I^T Ltil_J^T, so that sum_ij X_ij X_ji is
// an element-by-element product of the two (twice for I < J); a diagonal
// tile's own transpose is taken through the wavefront's LDS scratch instead
// of by two more products.  The next chunk's Ltil fragments are loaded while
// the current chunk's products run; TP: its Theta fragments are read from
// LDS ahead too.
template <bool X3, int NT, int NR, int ROLE, bool TP>
__device__ __forceinline__ void xch_waves(int wq, int KC, int G, long vsb,
                                          const afq_bf8* __restrict__ Lh,
                                          const afq_bf8* __restrict__ Ll, const afq_bf8* tfr,
                                          float* scr, double* __restrict__ vs_re,
                                          double* __restrict__ vs_im, double& xx_re,
                                          double& xx_im) {
  // role 0 of NR = 2: the diagonal pairs (two products each: X and, by an
  // LDS transposition, its own transpose) and about as many off-diagonal
  // pairs (four products each) as leave the two roles equal work
  constexpr int NPR = NT * (NT + 1) / 2;
  constexpr int NA = NR == 1 ? NPR : NT + (4 * (NPR - NT) - 2 * NT + 4) / 8;
  constexpr int LO = ROLE == 0 ? 0 : NA, HI = ROLE == 0 ? NA : NPR, NL = HI - LO;
  const int l = lane_id(), li = l & 15, lk = l >> 4;
  const int FR = NT * KC * 64;
  afq_bf8 a[NT], al[NT], br[NT], bi[NT], brl[NT], bil[NT];
  auto load_theta = [&](int kc, afq_bf8 (&r)[NT], afq_bf8 (&i)[NT], afq_bf8 (&rl)[NT],
                        afq_bf8 (&il)[NT]) __attribute__((always_inline)) {
#pragma unroll
    for (int J = 0; J < NT; ++J) {
      r[J] = tfr[(J * KC + kc) * 64 + l];
      i[J] = tfr[FR + (J * KC + kc) * 64 + l];
      if (X3) {
        rl[J] = tfr[2 * FR + (J * KC + kc) * 64 + l];
        il[J] = tfr[3 * FR + (J * KC + kc) * 64 + l];
      }
    }
  };
  if (wq < G) {
#pragma unroll
    for (int I = 0; I < NT; ++I) {
      a[I] = Lh[(long)wq * FR + I * KC * 64 + l];
      if (X3) al[I] = Ll[(long)wq * FR + I * KC * 64 + l];
    }
    if (TP) load_theta(0, br, bi, brl, bil);
  }
  for (int q = wq; q < G; q += 4) {
    afq_f4 acc[NL][4];
#pragma unroll
    for (int p = 0; p < NL; ++p)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[p][c] = afq_f4{0.f, 0.f, 0.f, 0.f};
    for (int kc = 0; kc < KC; ++kc) {
      int qn = q, kn = kc + 1;
      if (kn == KC) {
        kn = 0;
        qn = q + 4 < G ? q + 4 : q;
      }
      afq_bf8 an[NT], aln[NT];
#pragma unroll
      for (int I = 0; I < NT; ++I) {
        an[I] = Lh[(long)qn * FR + (I * KC + kn) * 64 + l];
        if (X3) aln[I] = Ll[(long)qn * FR + (I * KC + kn) * 64 + l];
      }
      afq_bf8 bnr[NT], bni[NT], bnrl[NT], bnil[NT];
      if (TP) load_theta(kn, bnr, bni, bnrl, bnil);
      else load_theta(kc, br, bi, brl, bil);
#pragma unroll
      for (int I = 0; I < NT; ++I)
#pragma unroll
        for (int J = I; J < NT; ++J) {
          const int gq = xch_pair(NT, I, J);
          if (gq < LO || gq >= HI) continue;
          const int p = gq - LO;
          if (X3) {
            acc[p][0] = mfma_bf16(al[I], br[J], acc[p][0]);
            acc[p][0] = mfma_bf16(a[I], brl[J], acc[p][0]);
            acc[p][1] = mfma_bf16(al[I], bi[J], acc[p][1]);
            acc[p][1] = mfma_bf16(a[I], bil[J], acc[p][1]);
            if (I != J) {
              acc[p][2] = mfma_bf16(brl[I], a[J], acc[p][2]);
              acc[p][2] = mfma_bf16(br[I], al[J], acc[p][2]);
              acc[p][3] = mfma_bf16(bil[I], a[J], acc[p][3]);
              acc[p][3] = mfma_bf16(bi[I], al[J], acc[p][3]);
            }
          }
          acc[p][0] = mfma_bf16(a[I], br[J], acc[p][0]);
          acc[p][1] = mfma_bf16(a[I], bi[J], acc[p][1]);
          if (I != J) {
            acc[p][2] = mfma_bf16(br[I], a[J], acc[p][2]);
            acc[p][3] = mfma_bf16(bi[I], a[J], acc[p][3]);
          }
        }
#pragma unroll
      for (int I = 0; I < NT; ++I) {
        a[I] = an[I];
        if (X3) al[I] = aln[I];
        if (TP) {
          br[I] = bnr[I];
          bi[I] = bni[I];
          brl[I] = bnrl[I];
          bil[I] = bnil[I];
        }
      }
    }
    // X_IJ and X^T_IJ hold X_ij and X_ji at the same place of the same lane
    float dr = 0.f, di = 0.f, orr = 0.f, oi = 0.f, tre = 0.f, tim = 0.f;
#pragma unroll
    for (int I = 0; I < NT; ++I)
#pragma unroll
      for (int J = I; J < NT; ++J) {
        const int gq = xch_pair(NT, I, J);
        if (gq < LO || gq >= HI) continue;
        const int p = gq - LO;
        if (I == J) {
          // X_II^T at the lane's places: X_II written as [row][col] (row
          // stride 20 floats: conflict-free writes, 16-byte aligned reads),
          // read back as [col][row]
          wave_lds_sync();
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            scr[(4 * lk + v) * 20 + li] = acc[p][0][v];
            scr[320 + (4 * lk + v) * 20 + li] = acc[p][1][v];
          }
          wave_lds_sync();
          acc[p][2] = *(const afq_f4*)(scr + li * 20 + 4 * lk);
          acc[p][3] = *(const afq_f4*)(scr + 320 + li * 20 + 4 * lk);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const float xr = acc[p][0][v], xi = acc[p][1][v], yr = acc[p][2][v], yi = acc[p][3][v];
          if (I == J) {
            dr += xr * yr - xi * yi;
            di += xr * yi + xi * yr;
            if (row_bf16(lk, v) == li) {
              tre += xr;
              tim += xi;
            }
          } else {
            orr += xr * yr - xi * yi;
            oi += xr * yi + xi * yr;
          }
        }
      }
    xx_re += (double)dr + 2.0 * (double)orr;
    xx_im += (double)di + 2.0 * (double)oi;
    if (ROLE == 0) {
      const double t_re = wave_sum((double)tre), t_im = wave_sum((double)tim);
      if (l == 0) {
        vs_re[vsb + q] = t_re;
        vs_im[vsb + q] = t_im;
      }
    }
  }
}

// Fused exchange (N_P <= 64, so at most four row tiles) with Ltil_g held in
// registers: one block per (walker, spin) stages Theta once in LDS in
// fragment order (hi, im and, X3, their second terms); four wavefronts (NR =
// 1) take every fourth g each with all tile pairs, or eight (NR = 2) split
// the pairs of each g in two halves between the two wavefronts of a SIMD,
// which halves their accumulators (the split form's operands and
// accumulators need over 256 registers for all pairs, so one wavefront per
// SIMD otherwise).
template <bool X3, int NT, int NR>
__global__ __launch_bounds__(256 * NR, (X3 || NR == 2) ? 1 : 2) void k_exchange_bf16_rf(
    int M, int KC, int Nt, int G, SpinGeom s0, SpinGeom s1, const afq_bf8* __restrict__ Ll0,
    const afq_bf8* __restrict__ Ll1, const double* __restrict__ thr,
    const double* __restrict__ thi, double* __restrict__ vs_re, double* __restrict__ vs_im,
    double* exx_re, double* exx_im) {
  extern __shared__ afq_bf8 tfr[];  // [X3 ? 4 : 2][NT][KC][64]
  __shared__ double red[16];
  const int w = blockIdx.x, s = blockIdx.y;
  const SpinGeom gm = s ? s1 : s0;
  const int N = gm.N, off = gm.off;
  const int wv = wave_id(), l = lane_id();
  if (N == 0) {
    for (int q = threadIdx.x; q < G; q += blockDim.x) {
      vs_re[((long)w * 2 + s) * G + q] = 0.0;
      vs_im[((long)w * 2 + s) * G + q] = 0.0;
    }
    if (threadIdx.x == 0) { exx_re[2 * w + s] = 0.0; exx_im[2 * w + s] = 0.0; }
    return;
  }
  const afq_bf8* __restrict__ Lh = (const afq_bf8*)gm.Lt;
  const afq_bf8* __restrict__ Ll = s ? Ll1 : Ll0;
  const int NP = 16 * NT, FR = NT * KC * 64;
  const long wb = (long)w * M * Nt;
  // fragment (J, kc, lane) of a component holds Theta[32 kc + 8 lk + e][16 J + li];
  // consecutive threads take consecutive columns so that the FP64 reads coalesce
  for (int f = threadIdx.x; f < NP * KC * 4; f += blockDim.x) {
    const int b = f % NP, mg = f / NP;
    afq_bf8 hr, hm, lr, lm;
    for (int e = 0; e < 8; ++e) {
      const int m = 8 * mg + e;
      const bool ok = m < M && b < N;
      const double xr = ok ? thr[wb + (long)m * Nt + off + b] : 0.0;
      const double xi = ok ? thi[wb + (long)m * Nt + off + b] : 0.0;
      hr[e] = (__bf16)(float)xr;
      hm[e] = (__bf16)(float)xi;
      if (X3) {
        lr[e] = bf16_lo(xr);
        lm[e] = bf16_lo(xi);
      }
    }
    const int at = ((b >> 4) * KC + (mg >> 2)) * 64 + (b & 15) + 16 * (mg & 3);
    tfr[at] = hr;
    tfr[FR + at] = hm;
    if (X3) {
      tfr[2 * FR + at] = lr;
      tfr[3 * FR + at] = lm;
    }
  }
  __syncthreads();
  double xx_re = 0.0, xx_im = 0.0;
  const long vsb = ((long)w * 2 + s) * G;
  // the wavefront's transposition scratch (2 x 16 x 20 floats) after Theta
  float* scr = (float*)(tfr + (X3 ? 4 : 2) * FR) + wv * 640;
  if constexpr (NR == 1) {
    // one wavefront per SIMD in the split form: Theta read ahead as well
    xch_waves<X3, NT, 1, 0, X3>(wv, KC, G, vsb, Lh, Ll, tfr, scr, vs_re, vs_im, xx_re, xx_im);
  } else {
    if (wv < 4)
      xch_waves<X3, NT, 2, 0, false>(wv, KC, G, vsb, Lh, Ll, tfr, scr, vs_re, vs_im, xx_re,
                                     xx_im);
    else
      xch_waves<X3, NT, 2, 1, false>(wv - 4, KC, G, vsb, Lh, Ll, tfr, scr, vs_re, vs_im, xx_re,
                                     xx_im);
  }
  xx_re = wave_sum(xx_re);
  xx_im = wave_sum(xx_im);
  if (l == 0) { red[wv] = xx_re; red[8 + wv] = xx_im; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double er = 0.0, ei = 0.0;
    for (int k = 0; k < 4 * NR; ++k) {
      er += red[k];
      ei += red[8 + k];
    }
    exx_re[2 * w + s] = er;
    exx_im[2 * w + s] = ei;
  }
}

hipError_t exchange_bf16(hipStream_t st, int W, int M, int MP32, int Nt, int G, SpinGeom s0,
                         SpinGeom s1, const void* Lt_lo0, const void* Lt_lo1, const double* thr,
                         const double* thi, double* vs_re, double* vs_im, double* exx_re,
                         double* exx_im, size_t max_lds) {
  const int NP = s0.NP > s1.NP ? s0.NP : s1.NP;
  const bool x3 = Lt_lo0 && Lt_lo1;
  const int KC = MP32 / 32;
  const afq_bf8 *l0 = (const afq_bf8*)Lt_lo0, *l1 = (const afq_bf8*)Lt_lo1;
  if (NP <= 64) {
    const int nrr = (x3 && NP > 32) ? 2 : 1;  // eight wavefronts per block for the split form's NT >= 3
    const size_t lds = (size_t)(x3 ? 4 : 2) * (NP / 16) * KC * 64 * sizeof(afq_bf8) +
                       (size_t)4 * nrr * 640 * sizeof(float);
    if (lds > max_lds) return hipErrorInvalidValue;
#define AFQ_XRF(X, NTT, NRR)                                                                       \
  hipLaunchKernelGGL((k_exchange_bf16_rf<X, NTT, NRR>), dim3(W, 2), dim3(256 * NRR), lds, st, M, KC, \
                     Nt, G, s0, s1, l0, l1, thr, thi, vs_re, vs_im, exx_re, exx_im)
    switch ((x3 ? 8 : 0) + NP / 16) {
      case 1: AFQ_XRF(false, 1, 1); break;
      case 2: AFQ_XRF(false, 2, 1); break;
      case 3: AFQ_XRF(false, 3, 1); break;
      case 4: AFQ_XRF(false, 4, 1); break;
      case 9: AFQ_XRF(true, 1, 1); break;
      case 10: AFQ_XRF(true, 2, 1); break;
      case 11: AFQ_XRF(true, 3, 2); break;
      case 12: AFQ_XRF(true, 4, 2); break;
      default: return hipErrorInvalidValue;
    }
#undef AFQ_XRF
    return hipGetLastError();
  }
  return hipErrorInvalidValue;  // N_P <= 64 always (at most 64 electrons per spin)
}

}  // namespace afq
