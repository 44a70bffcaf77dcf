// Walker-resident propagation (Sec. II step; walkers of several systems in
// one launch).  One workgroup owns one walker for a segment of K timesteps:
// its orbitals, propagator, Taylor terms, overlap inverses and force bias
// live in LDS, and so do the system's operators (L_g, B1 - I, D_0, the
// half-rotated Ltil_g, htil, lbar), staged once per segment from global
// memory (the kernel is for tiny systems, whose walker steps are too small to
// fill the chip one kernel launch per sub-step: the latency-bound regime).
// Each step is the one of the per-kernel chain:
//   fields x (Philox4x64-10 + Box-Muller, counter (t, walker, g/4, system)),
//   A = i sqrt(dt) sum_g (x_g - xbar_g) L_g with xbar = -i sqrt(dt)(v - lbar),
//   phi <- B1 exp(A) B1 phi (Taylor series), S = D_0^T phi per spin with its
//   inverse and log det (Gauss-Jordan, partial pivoting), Theta = phi S^-1,
//   E_L = e_core + sum Tr(htil Theta) + 1/2 sum_g (sum_s Tr X)^2
//         - 1/2 sum_s sum_g Tr(X X), X = Ltil_g Theta,
//   the phaseless weight, the dead-walker reset, and MGS every ortho_every
//   steps with log S recomputed.
// All arithmetic is FP64.  Every sum is taken in an order fixed by the
// problem (serial loops over a fixed index range, or per-item partials
// summed serially), never by the thread count, so a walker's results are
// bitwise the same for any block size and any group it runs in.
#include <math.h>

#include "common.hpp"
#include "resident.hpp"

namespace afq {

namespace {

// Member of walker block b (wave-uniform, so its fields are scalar loads).
__device__ inline int res_find_member(const ResMember* mem, int n_mem, int b) {
  int m = 0;
  for (int k = 1; k < n_mem; ++k)
    if (mem[k].wbase <= b) m = k;
  return __builtin_amdgcn_readfirstlane(m);
}

// Sum of n values x[i * stride] by one wavefront in an order fixed by n alone
// (lane l adds i = l, l + 64, ... in turn, then the 64 lanes by a fixed
// butterfly), whatever the block size; every lane gets the total.
__device__ inline double wave_fixed_sum(const double* x, int n, int stride) {
  double v = 0.0;
  for (int i = lane_id(); i < n; i += AFQ_WAVE) v += x[i * stride];
  return wave_sum(v);
}

// Out = In + B (In), B real [M][M], In complex [M][Nt], all in LDS.  (At the
// sizes this kernel takes, thread-per-element products are faster than FP64
// MFMA tiles, whose dependent chains leave one wavefront waiting.)
__device__ void res_apply_b1(int M, int Nt, const double* B, const double* Inr,
                             const double* Ini, double* Outr, double* Outi) {
  const int n = M * Nt;
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    const int i = e / Nt, c = e - i * Nt;
    const double* b = B + (long)i * M;
    double sr = 0.0, si = 0.0;
#pragma unroll 4
    for (int k = 0; k < M; ++k) {
      const double bk = b[k];
      sr = fma(bk, Inr[k * Nt + c], sr);
      si = fma(bk, Ini[k * Nt + c], si);
    }
    Outr[e] = Inr[e] + sr;
    Outi[e] = Ini[e] + si;
  }
}

// Out = alpha A In (A complex [M][M], In complex [M][Nt], all in LDS); Z += Out.
__device__ void res_taylor_term(int M, int Nt, const double* Ar, const double* Ai,
                                const double* Inr, const double* Ini, double* Outr, double* Outi,
                                double* Zr, double* Zi, double alpha) {
  const int n = M * Nt;
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    const int i = e / Nt, c = e - i * Nt;
    const double* ar = Ar + i * M;
    const double* ai = Ai + i * M;
    double sr = 0.0, si = 0.0;
#pragma unroll 4
    for (int k = 0; k < M; ++k) {
      const double xr = Inr[k * Nt + c], xi = Ini[k * Nt + c];
      sr = fma(ar[k], xr, sr);
      sr = fma(-ai[k], xi, sr);
      si = fma(ar[k], xi, si);
      si = fma(ai[k], xr, si);
    }
    sr *= alpha;
    si *= alpha;
    Outr[e] = sr;
    Outi[e] = si;
    Zr[e] += sr;
    Zi[e] += si;
  }
}

// In-place inverse of an N x N complex matrix (row-major in LDS) by one
// wavefront: Gauss-Jordan with partial pivoting (largest |S_ik|, lowest row
// on ties), rows swapped explicitly, columns unscrambled at the end.  Returns
// log det = sum log|pivot| + i arg(prod pivot / |pivot| * (-1)^swaps) in
// every lane (|det| kept as a mantissa and a power of two); non-finite when
// S is singular.
__device__ zdbl res_gj_inverse(int N, double* Sr, double* Si) {
  const int l = lane_id();
  double pm = 1.0, phr = 1.0, phi = 0.0;  // |det| = pm 2^pe, phase phr + i phi
  int pe = 0;
  int myp = l;  // lane k keeps the row swapped with row k at step k
  int np2 = 1;
  while (np2 < N) np2 <<= 1;
  for (int k = 0; k < N; ++k) {
    double key = -1.0;
    int idx = N;
    if (l >= k && l < N) {
      const double a = Sr[l * N + k], b = Si[l * N + k];
      key = a * a + b * b;
      idx = l;
    }
    for (int o = np2 >> 1; o >= 1; o >>= 1) {
      const double ok = __shfl_xor(key, o, AFQ_WAVE);
      const int oi = __shfl_xor(idx, o, AFQ_WAVE);
      if (ok > key || (ok == key && oi < idx)) { key = ok; idx = oi; }
    }
    const int p = __builtin_amdgcn_readfirstlane(idx < N ? idx : k);
    if (l == k) myp = p;
    if (p != k) {
      for (int j = l; j < N; j += AFQ_WAVE) {
        const double tr = Sr[k * N + j], ti = Si[k * N + j];
        Sr[k * N + j] = Sr[p * N + j];
        Si[k * N + j] = Si[p * N + j];
        Sr[p * N + j] = tr;
        Si[p * N + j] = ti;
      }
      phr = -phr;
      phi = -phi;
    }
    wave_lds_sync();
    const zdbl pv = {Sr[k * N + k], Si[k * N + k]};
    const double mag = sqrt(pv.re * pv.re + pv.im * pv.im);
    const double rm = 1.0 / mag;
    const double ur = pv.re * rm, ui = pv.im * rm;
    {
      int e;
      pm = frexp(pm * mag, &e);
      pe += e;
      const double nr = phr * ur - phi * ui, ni = phr * ui + phi * ur;
      phr = nr;
      phi = ni;
    }
    const zdbl inv = {ur * rm, -ui * rm};  // 1 / pivot
    wave_lds_sync();
    for (int j = l; j < N; j += AFQ_WAVE) {
      const zdbl x = (j == k) ? zdbl{1.0, 0.0} : zdbl{Sr[k * N + j], Si[k * N + j]};
      const zdbl y = zmul(x, inv);
      Sr[k * N + j] = y.re;
      Si[k * N + j] = y.im;
    }
    wave_lds_sync();
    if (l < N && l != k) {
      const zdbl f = {Sr[l * N + k], Si[l * N + k]};
      for (int j = 0; j < N; ++j) {
        const zdbl x = (j == k) ? zdbl{0.0, 0.0} : zdbl{Sr[l * N + j], Si[l * N + j]};
        const zdbl r = {Sr[k * N + j], Si[k * N + j]};
        Sr[l * N + j] = x.re - (f.re * r.re - f.im * r.im);
        Si[l * N + j] = x.im - (f.re * r.im + f.im * r.re);
      }
    }
    wave_lds_sync();
  }
  for (int k = N - 1; k >= 0; --k) {
    const int p = __builtin_amdgcn_readlane(myp, k);
    if (p != k && l < N) {
      const double tr = Sr[l * N + k], ti = Si[l * N + k];
      Sr[l * N + k] = Sr[l * N + p];
      Si[l * N + k] = Si[l * N + p];
      Sr[l * N + p] = tr;
      Si[l * N + p] = ti;
    }
    wave_lds_sync();
  }
  return zdbl{log(pm) + pe * 0.69314718055994530942, atan2(phi, phr)};
}

// The same inverse for N <= 8 with the rows in registers (lane i owns row
// i) and implicit pivoting: column k is eliminated with the unused row of
// largest |S_ik| (lowest row on ties), the pivot row broadcast by lane reads,
// no row exchanges and no LDS traffic until the end, where
// S^-1[k(i)][p(j)] = R[i][j] is written back (p(k): the pivot row of column k;
// k(i): the column row i was the pivot of).  log det as res_gj_inverse, with
// the sign of the pivot permutation from its inversion count.
constexpr int kGjRegMax = 8;
__device__ __noinline__ zdbl res_gj_inverse_reg(int N, double* Sr, double* Si) {
  constexpr int NR = kGjRegMax;
  const int l = lane_id();
  double xr[NR], xi[NR];
#pragma unroll
  for (int j = 0; j < NR; ++j) {
    const bool ok = l < N && j < N;
    xr[j] = ok ? Sr[l * N + j] : 0.0;
    xi[j] = ok ? Si[l * N + j] : 0.0;
  }
  double pm = 1.0, phr = 1.0, phi = 0.0;
  int pe = 0, used = 0, myk = 0, myp = 0;
  int np2 = 1;
  while (np2 < N) np2 <<= 1;
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    if (k >= N) break;
    double key = (l < N && !used) ? xr[k] * xr[k] + xi[k] * xi[k] : -1.0;
    int idx = l < N && !used ? l : 64;
    for (int o = np2 >> 1; o >= 1; o >>= 1) {
      const double ok2 = __shfl_xor(key, o, AFQ_WAVE);
      const int oi = __shfl_xor(idx, o, AFQ_WAVE);
      if (ok2 > key || (ok2 == key && oi < idx)) { key = ok2; idx = oi; }
    }
    const int p = __builtin_amdgcn_readfirstlane(idx);
    if (l == k) myp = p;
    const double pvr = __shfl(xr[k], p, AFQ_WAVE), pvi = __shfl(xi[k], p, AFQ_WAVE);
    const double mag = sqrt(pvr * pvr + pvi * pvi);
    const double rm = 1.0 / mag;
    const double ur = pvr * rm, ui = pvi * rm;
    {
      int e;
      pm = frexp(pm * mag, &e);
      pe += e;
      const double nr = phr * ur - phi * ui, ni = phr * ui + phi * ur;
      phr = nr;
      phi = ni;
    }
    const double ir = ur * rm, ii = -ui * rm;  // 1 / pivot
    const bool piv = l == p;
    if (piv) {
      used = 1;
      myk = k;
    }
    // f = S_lk / pivot for the other rows
    const double fr = xr[k] * ir - xi[k] * ii, fi = xr[k] * ii + xi[k] * ir;
#pragma unroll
    for (int j = 0; j < NR; ++j) {
      if (j >= N) break;
      // every lane reads the pivot row's entry before anyone changes it
      const double rr = __shfl(xr[j], p, AFQ_WAVE), ri = __shfl(xi[j], p, AFQ_WAVE);
      double nr, ni;
      if (j == k) {
        nr = piv ? ir : -fr;
        ni = piv ? ii : -fi;
      } else if (piv) {
        nr = xr[j] * ir - xi[j] * ii;
        ni = xr[j] * ii + xi[j] * ir;
      } else {
        nr = xr[j] - (fr * rr - fi * ri);
        ni = xi[j] - (fr * ri + fi * rr);
      }
      xr[j] = nr;
      xi[j] = ni;
    }
  }
  // sign of the pivot permutation k -> p(k): its inversion count
  int inv = 0;
  for (int k2 = 0; k2 < N; ++k2) {
    const int pk2 = __builtin_amdgcn_readlane(myp, k2);
    if (l < N && k2 > l && pk2 < myp) ++inv;
  }
  const double invd = wave_sum((double)inv);
  if (((long)invd) & 1) {
    phr = -phr;
    phi = -phi;
  }
  wave_lds_sync();
  if (l < N) {
#pragma unroll
    for (int j = 0; j < NR; ++j) {
      if (j < N) {
        const int pj = __builtin_amdgcn_readlane(myp, j);
        Sr[myk * N + pj] = xr[j];
        Si[myk * N + pj] = xi[j];
      }
    }
  }
  wave_lds_sync();
  return zdbl{log(pm) + pe * 0.69314718055994530942, atan2(phi, phr)};
}

// log det of both spins' overlaps S = D_0^T phi, inverses left in Y (spin 0
// at Y[0 .. n0^2), spin 1 after it).  Results in sc[0..3].
__device__ void res_overlaps(const ResMember& P, const ResLds& Lo, double* sm) {
  const int M = P.M, Nt = P.Nt;
  const double* phr = sm + Lo.ph_r;
  const double* phi = sm + Lo.ph_i;
  double* Yr = sm + Lo.Y_r;
  double* Yi = sm + Lo.Y_i;
  const int n0 = P.n0, n1 = P.n1;
  const int tot = n0 * n0 + n1 * n1;
  for (int e = threadIdx.x; e < tot; e += blockDim.x) {
    const int s = e < n0 * n0 ? 0 : 1;
    const int N = s ? n1 : n0, off = s ? n0 : 0;
    const int r = s ? e - n0 * n0 : e;
    const int a = r / N, b = r - a * N;
    double sr = 0.0, si = 0.0;
    for (int m = 0; m < M; ++m) {
      const double d = sm[Lo.D0 + m * Nt + off + a];
      sr = fma(d, phr[m * Nt + off + b], sr);
      si = fma(d, phi[m * Nt + off + b], si);
    }
    Yr[e] = sr;
    Yi[e] = si;
  }
  __syncthreads();
  const int wv = wave_id(), nwv = blockDim.x / AFQ_WAVE;
  for (int s = 0; s < 2; ++s) {
    const int N = s ? n1 : n0;
    if (wv != (nwv > 1 ? s : 0)) continue;
    zdbl ld = {0.0, 0.0};
    if (N > kGjRegMax) ld = res_gj_inverse(N, Yr + (s ? n0 * n0 : 0), Yi + (s ? n0 * n0 : 0));
    else if (N > 0) ld = res_gj_inverse_reg(N, Yr + (s ? n0 * n0 : 0), Yi + (s ? n0 * n0 : 0));
    if (lane_id() == 0) {
      sm[Lo.sc + 2 * s] = ld.re;
      sm[Lo.sc + 2 * s + 1] = ld.im;
    }
  }
  __syncthreads();
}

// Theta = phi S^-1 into X; E1 = sum_s Tr(htil Theta); the force-bias traces
// v'_g = sum_s Tr(Ltil_g Theta) into cf; E_K = -1/2 sum_s sum_g Tr(X X).
// Leaves E_L in sc[4..5], log S (sum of spins) in sc[6..7] and the finite
// flag of v' in sc[8].
__device__ void res_measure(const ResMember& P, const ResLds& Lo, double* sm) {
  const int M = P.M, Nt = P.Nt, G = P.G, n0 = P.n0, n1 = P.n1;
  res_overlaps(P, Lo, sm);
  const double* phr = sm + Lo.ph_r;
  const double* phi = sm + Lo.ph_i;
  double* Xr = sm + Lo.X_r;
  double* Xi = sm + Lo.X_i;
  const double* Yr = sm + Lo.Y_r;
  const double* Yi = sm + Lo.Y_i;
  // Theta[m][off + b] = sum_k phi[m][off + k] Sinv[k][b]
  for (int e = threadIdx.x; e < M * Nt; e += blockDim.x) {
    const int m = e / Nt, c = e - m * Nt;
    const int s = c < n0 ? 0 : 1;
    const int N = s ? n1 : n0, off = s ? n0 : 0, b = c - off;
    const double* Sr = Yr + (s ? n0 * n0 : 0);
    const double* Si = Yi + (s ? n0 * n0 : 0);
    double tr = 0.0, ti = 0.0;
    for (int k = 0; k < N; ++k) {
      const double ar = phr[m * Nt + off + k], ai = phi[m * Nt + off + k];
      const double br = Sr[k * N + b], bi = Si[k * N + b];
      tr = fma(ar, br, tr);
      tr = fma(-ai, bi, tr);
      ti = fma(ar, bi, ti);
      ti = fma(ai, br, ti);
    }
    Xr[e] = tr;
    Xi[e] = ti;
  }
  __syncthreads();
  // E1 partials per column (s, a): sum_m htil[a][m] Theta[m][off + a]
  double* red = sm + Lo.red;
  for (int c = threadIdx.x; c < Nt; c += blockDim.x) {
    const int s = c < n0 ? 0 : 1;
    const int a = c - (s ? n0 : 0);
    const double* h = sm + Lo.ht + c * M;
    double er = 0.0, ei = 0.0;
    for (int m = 0; m < M; ++m) {
      er = fma(h[m], Xr[m * Nt + c], er);
      ei = fma(h[m], Xi[m * Nt + c], ei);
    }
    red[2 * c] = er;
    red[2 * c + 1] = ei;
  }
  // exchange per spin: X_g = Ltil_g Theta for every g (rows (g, a) in
  // parallel), then per row the Tr X and Tr(X X) partials, then per g their
  // sums over rows
  double* trr = sm + Lo.tr_r;
  double* tri = sm + Lo.tr_i;
  double* xxr = sm + Lo.xx_r;
  double* xxi = sm + Lo.xx_i;
  double* Qr = sm + Lo.Xg_r;
  double* Qi = sm + Lo.Xg_i;
  double* ptr = sm + Lo.pt_r;
  double* pti = sm + Lo.pt_i;
  double* pxr = sm + Lo.px_r;
  double* pxi = sm + Lo.px_i;
  const int G1 = G > 0 ? G : 1;
  for (int s = 0; s < 2; ++s) {
    const int N = s ? n1 : n0, off = s ? n0 : 0;
    const double* Lt = sm + Lo.Lt + (s ? G * n0 * M : 0);  // [G][N][M]
    __syncthreads();
    if (N == 0) {
      for (int g = threadIdx.x; g < G; g += blockDim.x) {
        trr[s * G1 + g] = tri[s * G1 + g] = 0.0;
        xxr[s * G1 + g] = xxi[s * G1 + g] = 0.0;
      }
      continue;
    }
    // X for all g as one FP64 MFMA product: rows (g, a) of Ltil (k = m)
    // times Theta's spin columns, 16 x 16 output tiles over the wavefronts;
    // rows and columns past the ends are clamped (computed, never stored)
    {
      typedef Mfma<double> MM;
      const int R = G * N, RT = (R + 15) / 16, CT = (N + 15) / 16, KS = (M + 3) / 4;
      const int li = lane_id() & 15, lk = lane_id() >> 4;
      const int nwv = blockDim.x / AFQ_WAVE;
      for (int t = wave_id(); t < RT * CT; t += nwv) {
        const int rt = t / CT, ct = t - rt * CT;
        const int row = min(16 * rt + li, R - 1), colc = off + min(16 * ct + li, N - 1);
        MM::acc_t cr = MM::zero(), ci = MM::zero();
        for (int ks = 0; ks < KS; ++ks) {
          const int k = 4 * ks + lk, kc = min(k, M - 1);
          const double av = k < M ? Lt[row * M + kc] : 0.0;
          cr = MM::mma(av, Xr[kc * Nt + colc], cr);
          ci = MM::mma(av, Xi[kc * Nt + colc], ci);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = 16 * rt + MM::row(lk, v), c = 16 * ct + li;
          if (r < R && c < N) {
            Qr[r * N + c] = cr[v];
            Qi[r * N + c] = ci[v];
          }
        }
      }
    }
    __syncthreads();
    for (int task = threadIdx.x; task < G * N; task += blockDim.x) {
      const int g = task / N, a = task - g * N;
      const double* xr = Qr + g * N * N;
      const double* xi = Qi + g * N * N;
      double qr = 0.0, qi = 0.0;
      for (int b = 0; b < N; ++b) {
        const double ur = xr[a * N + b], ui = xi[a * N + b];
        const double vr = xr[b * N + a], vi = xi[b * N + a];
        qr += ur * vr - ui * vi;
        qi += ur * vi + ui * vr;
      }
      ptr[task] = xr[a * N + a];
      pti[task] = xi[a * N + a];
      pxr[task] = qr;
      pxi[task] = qi;
    }
    __syncthreads();
    for (int g = threadIdx.x; g < G; g += blockDim.x) {
      double tr = 0.0, ti = 0.0, qr = 0.0, qi = 0.0;
      for (int a = 0; a < N; ++a) {
        tr += ptr[g * N + a];
        ti += pti[g * N + a];
        qr += pxr[g * N + a];
        qi += pxi[g * N + a];
      }
      trr[s * G1 + g] = tr;
      tri[s * G1 + g] = ti;
      xxr[s * G1 + g] = qr;
      xxi[s * G1 + g] = qi;
    }
  }
  __syncthreads();
  double* cfr = sm + Lo.cf_r;
  double* cfi = sm + Lo.cf_i;
  for (int g = threadIdx.x; g < G; g += blockDim.x) {
    cfr[g] = trr[g] + trr[G1 + g];
    cfi[g] = tri[g] + tri[G1 + g];
  }
  __syncthreads();
  // the sums over g and over columns by wavefront 0, in fixed orders
  if (wave_id() == 0) {
    const double e1r = wave_fixed_sum(red, Nt, 2), e1i = wave_fixed_sum(red + 1, Nt, 2);
    double ejr = 0.0, eji = 0.0, ekr = 0.0, eki = 0.0, bad = 0.0;
    for (int g = lane_id(); g < G; g += AFQ_WAVE) {
      const double vr = cfr[g], vi = cfi[g];
      if (!isfinite(vr) || !isfinite(vi)) bad = 1.0;
      ejr += vr * vr - vi * vi;
      eji += 2.0 * vr * vi;
      ekr += xxr[g] + xxr[G1 + g];
      eki += xxi[g] + xxi[G1 + g];
    }
    ejr = wave_sum(ejr);
    eji = wave_sum(eji);
    ekr = wave_sum(ekr);
    eki = wave_sum(eki);
    bad = wave_sum(bad);
    if (lane_id() == 0) {
      double* sc = sm + Lo.sc;
      sc[4] = P.e_core + e1r + 0.5 * ejr - 0.5 * ekr;
      sc[5] = e1i + 0.5 * eji - 0.5 * eki;
      sc[6] = sc[0] + sc[2];
      sc[7] = sc[1] + sc[3];
      sc[8] = bad == 0.0 ? 1.0 : 0.0;
    }
  }
  __syncthreads();
}

// MGS of both spin blocks (one wavefront per spin, lane m owning row m),
// positive real diagonal of R.
__device__ void res_mgs(const ResMember& P, const ResLds& Lo, double* sm) {
  const int M = P.M, Nt = P.Nt;
  double* phr = sm + Lo.ph_r;
  double* phi = sm + Lo.ph_i;
  const int wv = wave_id(), nwv = blockDim.x / AFQ_WAVE, l = lane_id();
  for (int s = 0; s < 2; ++s) {
    if (wv != (nwv > 1 ? s : 0)) continue;
    const int N = s ? P.n1 : P.n0, off = s ? P.n0 : 0;
    for (int j = 0; j < N; ++j) {
      double qr = l < M ? phr[l * Nt + off + j] : 0.0;
      double qi = l < M ? phi[l * Nt + off + j] : 0.0;
      const double nrm = sqrt(wave_sum(qr * qr + qi * qi));
      const double inv = 1.0 / nrm;
      qr *= inv;
      qi *= inv;
      if (l < M) {
        phr[l * Nt + off + j] = qr;
        phi[l * Nt + off + j] = qi;
      }
      for (int k = j + 1; k < N; ++k) {
        double ar = l < M ? phr[l * Nt + off + k] : 0.0;
        double ai = l < M ? phi[l * Nt + off + k] : 0.0;
        const double rr = wave_sum(qr * ar + qi * ai);
        const double ri = wave_sum(qr * ai - qi * ar);
        ar -= rr * qr - ri * qi;
        ai -= rr * qi + ri * qr;
        if (l < M) {
          phr[l * Nt + off + k] = ar;
          phi[l * Nt + off + k] = ai;
        }
      }
    }
  }
  __syncthreads();
}

}  // namespace

__global__ __launch_bounds__(512) void k_res_steps(const ResMember* __restrict__ mem, int n_mem,
                                                   int w_total, const uint64_t* __restrict__ tdev,
                                                   int K, int refresh, double* __restrict__ wsum) {
  extern __shared__ double sm[];
  const int b = blockIdx.x;
  const ResMember& P = mem[res_find_member(mem, n_mem, b)];
  const int w = b - P.wbase;
  const int M = P.M, Nt = P.Nt, G = P.G, mn = M * Nt;
  const ResLds Lo = res_lds(M, Nt, G, P.n0 > P.n1 ? P.n0 : P.n1);
  double* phr = sm + Lo.ph_r;
  double* phi = sm + Lo.ph_i;
  double* vr = sm + Lo.v_r;
  double* vi = sm + Lo.v_i;
  double* sc = sm + Lo.sc;
  for (int e = threadIdx.x; e < mn; e += blockDim.x) {
    phr[e] = P.phi_re[(long)w * mn + e];
    phi[e] = P.phi_im[(long)w * mn + e];
  }
  for (int g = threadIdx.x; g < G; g += blockDim.x) {
    vr[g] = P.v_re[(long)w * G + g];
    vi[g] = P.v_im[(long)w * G + g];
  }
  // the member's operators, once per segment
  {
    const int mm = M * M, n0 = P.n0, n1 = P.n1;
    for (int e = threadIdx.x; e < mm; e += blockDim.x) sm[Lo.B1 + e] = P.B1m[e];
    for (int e = threadIdx.x; e < mn; e += blockDim.x) {
      sm[Lo.D0 + e] = P.D0[e];
      const int c = e / M, m = e - c * M;
      sm[Lo.ht + e] = c < n0 ? P.ht0[c * M + m] : P.ht1[(c - n0) * M + m];
    }
    for (int g = threadIdx.x; g < G; g += blockDim.x) sm[Lo.lb + g] = P.lbar[g];
    for (int e = threadIdx.x; e < G * mn; e += blockDim.x) {
      // spin 0: [G][n0][M] from Ltil[(g MP4 + m) NP0 + a]; then spin 1
      const int s1 = e >= G * n0 * M;
      const int r = s1 ? e - G * n0 * M : e;
      const int N = s1 ? n1 : n0;
      const int g = r / (N * M), q = r - g * N * M, a = q / M, m = q - a * M;
      sm[Lo.Lt + e] = s1 ? P.Lt1[((long)g * P.MP4 + m) * P.NP1 + a]
                         : P.Lt0[((long)g * P.MP4 + m) * P.NP0 + a];
    }
    for (long e = threadIdx.x; e < (long)G * mm; e += blockDim.x) sm[Lo.L + e] = P.L[e];
  }
  // walker scalars: sc[16..21] = weight, log S (re, im), E_L (re, im)
  if (threadIdx.x == 0) {
    sc[16] = P.weight[w];
    sc[17] = P.ls_re[w];
    sc[18] = P.ls_im[w];
    sc[19] = P.el_re[w];
    sc[20] = P.el_im[w];
  }
  __syncthreads();
  if (refresh) {
    res_measure(P, Lo, sm);
    for (int g = threadIdx.x; g < G; g += blockDim.x) {
      vr[g] = sm[Lo.cf_r + g];
      vi[g] = sm[Lo.cf_i + g];
    }
    if (threadIdx.x == 0) {
      sc[17] = sc[6];
      sc[18] = sc[7];
      sc[19] = sc[4];
      sc[20] = sc[5];
    }
    __syncthreads();
  }
  const uint64_t t0 = K > 0 ? *tdev : 0;
  const double sq = P.sqdt;
  double* cfr = sm + Lo.cf_r;
  double* cfi = sm + Lo.cf_i;
  double* red = sm + Lo.red;
  double* Ar = sm + Lo.A_r;
  double* Ai = sm + Lo.A_i;
  double* Xr = sm + Lo.X_r;
  double* Xi = sm + Lo.X_i;
  double* Yr = sm + Lo.Y_r;
  double* Yi = sm + Lo.Y_i;
  double* Zr = sm + Lo.Z_r;
  double* Zi = sm + Lo.Z_i;
  for (int s = 0; s < K; ++s) {
    const uint64_t t = t0 + (uint64_t)s;
    // fields, shifted coefficients xs = x - xbar and the mean-field log factor
    const int nq = (G + 3) / 4;
    for (int q = threadIdx.x; q < nq; q += blockDim.x) {
      double z[4];
      gaussian4(P.seed, t, (uint64_t)w, (uint64_t)q, (uint64_t)P.system_id, z);
      double pr = 0.0, pi = 0.0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int g = 4 * q + j;
        if (g < G) {
          const double lb = sm[Lo.lb + g];
          const double xsr = z[j] - sq * vi[g];
          const double xsi = sq * (vr[g] - lb);
          cfr[g] = xsr;
          cfi[g] = xsi;
          pr += sq * xsi * lb;
          pi += -sq * xsr * lb;
        }
      }
      red[2 * q] = pr;
      red[2 * q + 1] = pi;
    }
    __syncthreads();
    if (wave_id() == 0) {
      const double mr = wave_fixed_sum(red, nq, 2), mi = wave_fixed_sum(red + 1, nq, 2);
      if (lane_id() == 0) {
        sc[10] = mr;
        sc[11] = mi;
      }
    }
    // A = i sq sum_g xs_g L_g (symmetric): upper triangle, mirrored
    for (int e = threadIdx.x; e < M * M; e += blockDim.x) {
      const int i = e / M, j = e - i * M;
      if (i > j) continue;
      double ar = 0.0, ai = 0.0;
      const double* l = sm + Lo.L + e;
      for (int g = 0; g < G; ++g) {
        const double lv = l[g * M * M];
        ar = fma(cfi[g], lv, ar);
        ai = fma(cfr[g], lv, ai);
      }
      ar *= -sq;
      ai *= sq;
      Ar[e] = ar;
      Ai[e] = ai;
      Ar[j * M + i] = ar;
      Ai[j * M + i] = ai;
    }
    // X = B1 phi
    res_apply_b1(M, Nt, sm + Lo.B1, phr, phi, Xr, Xi);
    __syncthreads();
    for (int e = threadIdx.x; e < mn; e += blockDim.x) {
      Zr[e] = Xr[e];
      Zi[e] = Xi[e];
    }
    __syncthreads();
    double* cr = Xr;
    double* ci = Xi;
    double* nr = Yr;
    double* ni = Yi;
    for (int n = 1; n <= P.order; ++n) {
      res_taylor_term(M, Nt, Ar, Ai, cr, ci, nr, ni, Zr, Zi, 1.0 / n);
      __syncthreads();
      double* tr = cr;
      double* ti = ci;
      cr = nr;
      ci = ni;
      nr = tr;
      ni = ti;
    }
    // phi = B1 ACC
    res_apply_b1(M, Nt, sm + Lo.B1, Zr, Zi, phr, phi);
    __syncthreads();
    res_measure(P, Lo, sm);
    // phaseless weight (local-energy form), dead-walker reset
    if (threadIdx.x == 0) {
      const double er = sc[4], ei = sc[5];
      const double lr = sc[6] - sc[17] + sc[10];
      const double li = sc[7] - sc[18] + sc[11];
      const double c = cos(li);
      const double wn = sc[16] * exp(-P.dt * (er - P.e_trial)) * (c > 0.0 ? c : 0.0);
      const bool ok = isfinite(wn) && isfinite(er) && isfinite(ei) && isfinite(lr) &&
                      isfinite(li) && isfinite(sc[6]) && isfinite(sc[7]) && sc[8] != 0.0 &&
                      wn > 0.0;
      if (ok) {
        sc[16] = wn;
        sc[17] = sc[6];
        sc[18] = sc[7];
        sc[19] = er;
        sc[20] = ei;
      } else {
        sc[16] = 0.0;
        sc[17] = P.ref_ls_re;
        sc[18] = P.ref_ls_im;
        sc[19] = P.ref_el_re;
        sc[20] = P.ref_el_im;
      }
      sc[12] = ok ? 1.0 : 0.0;
      const long o = ((long)s * w_total + b) * 2;
      wsum[o] = sc[16] * sc[19];
      wsum[o + 1] = sc[16];
    }
    __syncthreads();
    const bool alive = sc[12] != 0.0;
    for (int g = threadIdx.x; g < G; g += blockDim.x) {
      vr[g] = alive ? cfr[g] : P.vref_re[g];
      vi[g] = alive ? cfi[g] : P.vref_im[g];
    }
    if (!alive)
      for (int e = threadIdx.x; e < mn; e += blockDim.x) {
        phr[e] = sm[Lo.D0 + e];
        phi[e] = 0.0;
      }
    __syncthreads();
    if (P.ortho_every > 0 && (t + 1) % (uint64_t)P.ortho_every == 0) {
      res_mgs(P, Lo, sm);
      res_overlaps(P, Lo, sm);
      if (threadIdx.x == 0) {
        sc[17] = sc[0] + sc[2];
        sc[18] = sc[1] + sc[3];
      }
      __syncthreads();
    }
  }
  for (int e = threadIdx.x; e < mn; e += blockDim.x) {
    P.phi_re[(long)w * mn + e] = phr[e];
    P.phi_im[(long)w * mn + e] = phi[e];
  }
  for (int g = threadIdx.x; g < G; g += blockDim.x) {
    P.v_re[(long)w * G + g] = vr[g];
    P.v_im[(long)w * G + g] = vi[g];
  }
  if (threadIdx.x == 0) {
    P.weight[w] = sc[16];
    P.ls_re[w] = sc[17];
    P.ls_im[w] = sc[18];
    P.el_re[w] = sc[19];
    P.el_im[w] = sc[20];
  }
}

hipError_t res_steps(hipStream_t st, const ResMember* mem, int n_mem, int w_total, int threads,
                     size_t lds_bytes, const uint64_t* tdev, int K, int refresh, double* wsum) {
  if (w_total < 1) return hipSuccess;
  hipLaunchKernelGGL(k_res_steps, dim3(w_total), dim3(threads), lds_bytes, st, mem, n_mem, w_total,
                     tdev, K, refresh, wsum);
  return hipGetLastError();
}

// E_mix of every member and step of a segment: block (member, step), the
// member's walkers summed in a fixed order (256 threads, block_sum).
__global__ __launch_bounds__(256) void k_res_emix(const ResMember* __restrict__ mem, int w_total,
                                                  const uint64_t* __restrict__ tdev,
                                                  const double* __restrict__ wsum) {
  __shared__ double red[4];
  const ResMember& P = mem[blockIdx.x];
  const int s = blockIdx.y;
  if (!P.emix) return;
  double num = 0.0, den = 0.0;
  for (int w = threadIdx.x; w < P.W; w += blockDim.x) {
    const long o = ((long)s * w_total + P.wbase + w) * 2;
    num += wsum[o];
    den += wsum[o + 1];
  }
  num = block_sum(num, red);
  den = block_sum(den, red);
  if (threadIdx.x == 0) P.emix[(long)(*tdev + (uint64_t)s - P.call_step0)] = num / den;
}

hipError_t res_emix(hipStream_t st, const ResMember* mem, int n_mem, int w_total,
                    const uint64_t* tdev, int K, const double* wsum) {
  if (K < 1 || n_mem < 1) return hipSuccess;
  hipLaunchKernelGGL(k_res_emix, dim3(n_mem, K), dim3(256), 0, st, mem, w_total, tdev, wsum);
  return hipGetLastError();
}

// The systematic comb of a member whose comb falls at the end of the segment
// (after step t with (t + 1) % pc_every == 0): one block per member, the same
// algorithm as the single-system comb (left-to-right prefix sums in one
// thread, tooth j at ((j + xi) W_tot) / K, first walker whose prefix exceeds
// it); no teeth when W_tot is not positive and finite.
__global__ __launch_bounds__(1024) void k_res_comb_parents(const ResMember* __restrict__ mem,
                                                           const uint64_t* __restrict__ tdev,
                                                           int K) {
  __shared__ double sh[3];
  __shared__ int last_sh;
  const ResMember& P = mem[blockIdx.x];
  const uint64_t tl = *tdev + (uint64_t)K - 1;
  const bool due = P.pc_every > 0 && (tl + 1) % (uint64_t)P.pc_every == 0;
  const int W = P.W;
  if (threadIdx.x == 0) {
    double acc = 0.0;
    int last = W - 1;
    if (due)
      for (int k = 0; k < W; ++k) {
        const double wk = P.weight[k];
        if (wk > 0.0) last = k;
        acc = acc + wk;
        P.cbuf[k] = acc;
      }
    const PhiloxOut r = philox4x64_10(tl, 0ull, 0ull, (uint64_t)P.system_id, P.seed, AFQ_STREAM_COMB);
    sh[0] = acc;
    sh[1] = u64_to_unit(r.w[0]);
    sh[2] = (due && acc > 0.0 && isfinite(acc)) ? 1.0 : 0.0;
    last_sh = last;
    P.comb_scal[0] = due ? acc / (double)W : 0.0;
    P.comb_scal[1] = sh[2];
  }
  __syncthreads();
  if (sh[2] == 0.0) return;
  const double wtot = sh[0], xi = sh[1];
  const int last = last_sh;
  for (int j = threadIdx.x; j < W; j += blockDim.x) {
    const double zj = (((double)j + xi) * wtot) / (double)W;
    int lo = 0, hi = W;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (P.cbuf[mid] > zj) hi = mid; else lo = mid + 1;
    }
    P.parent[j] = (lo < W) ? lo : last;
  }
}

// Snapshot (phase 0) or gather from the parents (phase 1) of one walker of a
// combing member: orbitals, log S, E_L and the force-bias traces.
__global__ __launch_bounds__(256) void k_res_comb_move(const ResMember* __restrict__ mem, int n_mem,
                                                       int phase) {
  const int b = blockIdx.x;
  const ResMember& P = mem[res_find_member(mem, n_mem, b)];
  if (P.comb_scal[1] == 0.0) return;
  const int w = b - P.wbase;
  const long mn = (long)P.M * P.Nt, G = P.G, row = 2 * mn + 4 + 2 * G;
  if (phase == 0) {
    double* d = P.snap + w * row;
    for (long e = threadIdx.x; e < mn; e += blockDim.x) {
      d[e] = P.phi_re[w * mn + e];
      d[mn + e] = P.phi_im[w * mn + e];
    }
    for (long g = threadIdx.x; g < G; g += blockDim.x) {
      d[2 * mn + 4 + g] = P.v_re[w * G + g];
      d[2 * mn + 4 + G + g] = P.v_im[w * G + g];
    }
    if (threadIdx.x == 0) {
      d[2 * mn] = P.ls_re[w];
      d[2 * mn + 1] = P.ls_im[w];
      d[2 * mn + 2] = P.el_re[w];
      d[2 * mn + 3] = P.el_im[w];
    }
  } else {
    const double* s = P.snap + (long)P.parent[w] * row;
    for (long e = threadIdx.x; e < mn; e += blockDim.x) {
      P.phi_re[w * mn + e] = s[e];
      P.phi_im[w * mn + e] = s[mn + e];
    }
    for (long g = threadIdx.x; g < G; g += blockDim.x) {
      P.v_re[w * G + g] = s[2 * mn + 4 + g];
      P.v_im[w * G + g] = s[2 * mn + 4 + G + g];
    }
    if (threadIdx.x == 0) {
      P.ls_re[w] = s[2 * mn];
      P.ls_im[w] = s[2 * mn + 1];
      P.el_re[w] = s[2 * mn + 2];
      P.el_im[w] = s[2 * mn + 3];
      P.weight[w] = 1.0;
    }
  }
}

hipError_t res_comb(hipStream_t st, const ResMember* mem, int n_mem, int w_total,
                    const uint64_t* tdev, int K, int w_max) {
  if (K < 1 || n_mem < 1 || w_total < 1) return hipSuccess;
  (void)w_max;
  hipLaunchKernelGGL(k_res_comb_parents, dim3(n_mem), dim3(1024), 0, st, mem, tdev, K);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_res_comb_move, dim3(w_total), dim3(256), 0, st, mem, n_mem, 0);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_res_comb_move, dim3(w_total), dim3(256), 0, st, mem, n_mem, 1);
  return hipGetLastError();
}

__global__ void k_res_advance(uint64_t* tdev, int K) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *tdev += (uint64_t)K;
}

hipError_t res_advance(hipStream_t st, uint64_t* tdev, int K) {
  hipLaunchKernelGGL(k_res_advance, dim3(1), dim3(64), 0, st, tdev, K);
  return hipGetLastError();
}

struct ResCallArgs {
  uint64_t step0;
  int n_mem;
  double* emix[kResMaxMembers];
};

__global__ void k_res_begin(ResMember* mem, uint64_t* tdev, ResCallArgs a) {
  const int m = threadIdx.x;
  if (m < a.n_mem) {
    mem[m].call_step0 = a.step0;
    mem[m].emix = a.emix[m];
  }
  if (m == 0) *tdev = a.step0;
}

hipError_t res_begin(hipStream_t st, ResMember* mem, int n_mem, uint64_t* tdev, uint64_t step0,
                     double* const* emix) {
  if (n_mem < 1 || n_mem > kResMaxMembers) return hipErrorInvalidValue;
  ResCallArgs a;
  a.step0 = step0;
  a.n_mem = n_mem;
  for (int m = 0; m < kResMaxMembers; ++m) a.emix[m] = m < n_mem ? emix[m] : nullptr;
  hipLaunchKernelGGL(k_res_begin, dim3(1), dim3(kResMaxMembers), 0, st, mem, tdev, a);
  return hipGetLastError();
}

}  // namespace afq
