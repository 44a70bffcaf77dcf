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

// dst[r][c] = src[c][r] (src rows x cols FP64 -> bf16), batched over z;
// dst_lo (nullable) receives the split's second term.
__global__ void k_transpose_bf16(int rows, int cols, int ld_dst, long s_src, long s_dst,
                                 const double* src, __bf16* dst, __bf16* dst_lo) {
  const long z = blockIdx.z;
  const int c = blockIdx.x * 16 + (threadIdx.x & 15);
  const int r = blockIdx.y * 16 + (threadIdx.x >> 4);
  if (r < rows && c < cols) {
    const double x = src[z * s_src + (long)r * cols + c];
    dst[z * s_dst + (long)c * ld_dst + r] = (__bf16)(float)x;
    if (dst_lo) dst_lo[z * s_dst + (long)c * ld_dst + r] = bf16_lo(x);
  }
}

hipError_t transpose_f64_bf16(hipStream_t st, int rows, int cols, int ld_dst, long s_src,
                              long s_dst, int batch, const double* src, void* dst, void* dst_lo) {
  dim3 grid((cols + 15) / 16, (rows + 15) / 16, batch);
  hipLaunchKernelGGL(k_transpose_bf16, grid, dim3(256), 0, st, rows, cols, ld_dst, s_src, s_dst, src,
                     (__bf16*)dst, (__bf16*)dst_lo);
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

// Fused exchange in bf16: X_g = Ltil_g Theta with Ltil stored [g][a][MP32]
// (m contiguous) and Theta staged in LDS as [b][MP32] bf16; same tile pairing
// and reductions as the FP32/FP64 kernel.  X3: both operands split in two
// bf16 terms, three products per tile (the lo-lo one dropped), FP32
// accumulation.
template <bool X3>
__global__ __launch_bounds__(256) void k_exchange_bf16(int M, int MP32, int Nt, int G, SpinGeom s0,
                                                       SpinGeom s1, const __bf16* __restrict__ Ltl0,
                                                       const __bf16* __restrict__ Ltl1,
                                                       const double* __restrict__ thr,
                                                       const double* __restrict__ thi,
                                                       double* __restrict__ vs_re,
                                                       double* __restrict__ vs_im, double* exx_re,
                                                       double* exx_im) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_bf[];
  __shared__ double red[8];
  const int w = blockIdx.x, s = blockIdx.y;
  const SpinGeom g = s ? s1 : s0;
  const int N = g.N, NP = g.NP, off = g.off;
  const __bf16* __restrict__ Lt = (const __bf16*)g.Lt;
  const int wv = wave_id(), l = lane_id(), li = l & 15, lk = l >> 4;
  if (N == 0) {
    for (int q = threadIdx.x; q < G; q += blockDim.x) {
      vs_re[((long)w * 2 + s) * G + q] = 0.0;
      vs_im[((long)w * 2 + s) * G + q] = 0.0;
    }
    if (threadIdx.x == 0) { exx_re[2 * w + s] = 0.0; exx_im[2 * w + s] = 0.0; }
    return;
  }
  const __bf16* __restrict__ Ltl = s ? Ltl1 : Ltl0;
  __bf16* Tr = (__bf16*)lds_bf;          // [NP][MP32]
  __bf16* Ti = Tr + NP * MP32;
  __bf16* Trl = Ti + NP * MP32;          // X3: second terms
  __bf16* Til = Trl + (X3 ? NP * MP32 : 0);
  float* scr = (float*)(Til + (X3 ? NP * MP32 : 0));  // 4 waves x 2 x 256
  float* myr = scr + wv * 512;
  float* myi = myr + 256;
  const long wb = (long)w * M * Nt;
  const __bf16 zero = (__bf16)0.0f;
  for (int e = threadIdx.x; e < NP * MP32; e += blockDim.x) {
    const int b = e / MP32, m = e % MP32;
    const bool ok = m < M && b < N;
    const double xr = ok ? thr[wb + (long)m * Nt + off + b] : 0.0;
    const double xi = ok ? thi[wb + (long)m * Nt + off + b] : 0.0;
    Tr[e] = ok ? (__bf16)(float)xr : zero;
    Ti[e] = ok ? (__bf16)(float)xi : zero;
    if (X3) {
      Trl[e] = ok ? bf16_lo(xr) : zero;
      Til[e] = ok ? bf16_lo(xi) : zero;
    }
  }
  __syncthreads();
  const int NT = NP / 16;
  double xx_re = 0.0, xx_im = 0.0;
  for (int q = wv; q < G; q += 4) {
    const __bf16* Lq = Lt + (long)q * NP * MP32;
    double tr_re = 0.0, tr_im = 0.0;
    for (int I = 0; I < NT; ++I) {
      for (int J = I; J < NT; ++J) {
        afq_f4 pr = {0, 0, 0, 0}, pi = {0, 0, 0, 0}, qr = {0, 0, 0, 0}, qi = {0, 0, 0, 0};
        for (int k = 0; k < MP32; k += 32) {
          const afq_bf8 aI = *(const afq_bf8*)&Lq[(long)(16 * I + li) * MP32 + k + 8 * lk];
          const afq_bf8 bJr = *(const afq_bf8*)&Tr[(16 * J + li) * MP32 + k + 8 * lk];
          const afq_bf8 bJi = *(const afq_bf8*)&Ti[(16 * J + li) * MP32 + k + 8 * lk];
          if (X3) {
            const __bf16* Lql = Ltl + (long)q * NP * MP32;
            const afq_bf8 aIl = *(const afq_bf8*)&Lql[(long)(16 * I + li) * MP32 + k + 8 * lk];
            const afq_bf8 bJrl = *(const afq_bf8*)&Trl[(16 * J + li) * MP32 + k + 8 * lk];
            const afq_bf8 bJil = *(const afq_bf8*)&Til[(16 * J + li) * MP32 + k + 8 * lk];
            pr = mfma_bf16(aIl, bJr, pr);
            pr = mfma_bf16(aI, bJrl, pr);
            pi = mfma_bf16(aIl, bJi, pi);
            pi = mfma_bf16(aI, bJil, pi);
          }
          pr = mfma_bf16(aI, bJr, pr);
          pi = mfma_bf16(aI, bJi, pi);
          if (I != J) {
            const afq_bf8 aJ = *(const afq_bf8*)&Lq[(long)(16 * J + li) * MP32 + k + 8 * lk];
            const afq_bf8 bIr = *(const afq_bf8*)&Tr[(16 * I + li) * MP32 + k + 8 * lk];
            const afq_bf8 bIi = *(const afq_bf8*)&Ti[(16 * I + li) * MP32 + k + 8 * lk];
            if (X3) {
              const __bf16* Lql = Ltl + (long)q * NP * MP32;
              const afq_bf8 aJl = *(const afq_bf8*)&Lql[(long)(16 * J + li) * MP32 + k + 8 * lk];
              const afq_bf8 bIrl = *(const afq_bf8*)&Trl[(16 * I + li) * MP32 + k + 8 * lk];
              const afq_bf8 bIil = *(const afq_bf8*)&Til[(16 * I + li) * MP32 + k + 8 * lk];
              qr = mfma_bf16(aJl, bIr, qr);
              qr = mfma_bf16(aJ, bIrl, qr);
              qi = mfma_bf16(aJl, bIi, qi);
              qi = mfma_bf16(aJ, bIil, qi);
            }
            qr = mfma_bf16(aJ, bIr, qr);
            qi = mfma_bf16(aJ, bIi, qi);
          }
        }
        for (int v = 0; v < 4; ++v) {
          const int r = row_bf16(lk, v);
          myr[r * 16 + li] = (I != J) ? qr[v] : pr[v];
          myi[r * 16 + li] = (I != J) ? qi[v] : pi[v];
        }
        wave_lds_sync();
        const double mult = (I != J) ? 2.0 : 1.0;
        for (int v = 0; v < 4; ++v) {
          const int r = row_bf16(lk, v);
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

hipError_t exchange_bf16(hipStream_t st, int W, int M, int MP32, int Nt, int G, SpinGeom s0,
                         SpinGeom s1, const void* Lt_lo0, const void* Lt_lo1, const double* thr,
                         const double* thi, double* vs_re, double* vs_im, double* exx_re,
                         double* exx_im, size_t max_lds) {
  const int NP = s0.NP > s1.NP ? s0.NP : s1.NP;
  const bool x3 = Lt_lo0 && Lt_lo1;
  const size_t lds = (size_t)(x3 ? 4 : 2) * NP * MP32 * 2 + (size_t)4 * 512 * 4;
  if (lds > max_lds) return hipErrorInvalidValue;
  if (x3)
    hipLaunchKernelGGL(k_exchange_bf16<true>, dim3(W, 2), dim3(256), lds, st, M, MP32, Nt, G, s0, s1,
                       (const __bf16*)Lt_lo0, (const __bf16*)Lt_lo1, thr, thi, vs_re, vs_im, exx_re,
                       exx_im);
  else
    hipLaunchKernelGGL(k_exchange_bf16<false>, dim3(W, 2), dim3(256), lds, st, M, MP32, Nt, G, s0,
                       s1, nullptr, nullptr, thr, thi, vs_re, vs_im, exx_re, exx_im);
  return hipGetLastError();
}

}  // namespace afq
