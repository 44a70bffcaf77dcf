// gfx950 kernels of the Q route of the local energy (arXiv 1804.03310,
// Sec. III, Eq. Ys): the force bias as one GEMM over all walkers and the
// exchange sum_g Tr(X_g X_g) as the quadratic form theta^T Q theta per spin,
// with Q[(n a)][(m b)] = sum_g Ltil_g[a][m] Ltil_g[b][n] symmetric, so only
// tile pairs I <= J are visited (off-diagonal pairs count twice).
//
// Operand layout shared by both contraction kernels: per walker the split
// Theta row ts[w][0 .. Ktot) written by the overlap kernels, spin 0's M N_up
// entries (n a) -> n N_up + a first, zero padded to Kp0 = 64 ceil(M N_up /
// 64), then spin 1's.  A
// 16 x 16 x 4 MFMA step takes lane (i, q) = (l % 16, l / 16) -> walker i and
// k = 16 u + 4 q + j for the step (u, j), so each lane fetches its k values
// as one 4-vector; B is read from LDS with the same k order and the column
// of lane li being 4 li + jb for the four column tiles jb (one 4-vector).
#include "common.hpp"
#include "kernels.hpp"

namespace afq {

namespace {

template <typename T> struct V4;
template <> struct V4<float> { typedef float type __attribute__((ext_vector_type(4))); };
template <> struct V4<double> { typedef double type __attribute__((ext_vector_type(4))); };

// Row groups of 16 per wave in the A-build: one (at the headline size two
// groups per wave left the launch at 1.25 blocks per CU; one group gives
// twice the blocks and measured faster).
template <typename T> struct QGeom {
  static constexpr int GW = 1;
};

constexpr int QT = 64;       // tile edge along k and along the output columns
constexpr int QLD = QT + 4;  // LDS row stride (elements)

// Stage the 64 x 64 tile at (row r0, column c0) of a row-major matrix with
// leading dimension ld into registers: 16 elements per thread of 256.
template <typename T>
__device__ inline void tile_fetch(const T* __restrict__ A, long ld, long r0, long c0,
                                  typename V4<T>::type (&pre)[4]) {
  typedef typename V4<T>::type t4;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int idx = e * 256 + threadIdx.x, row = idx >> 4, c4 = idx & 15;
    pre[e] = *(const t4*)(A + (r0 + row) * ld + c0 + 4 * c4);
  }
}

// PAIRS: columns 4 c + jb stored at (jb / 2) 32 + 2 c + jb % 2, so that the
// two-column passes of the quadratic form read 8 contiguous bytes per lane.
template <typename T, bool PAIRS>
__device__ inline void tile_store(T* lds, const typename V4<T>::type (&pre)[4]) {
  typedef typename V4<T>::type t4;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int idx = e * 256 + threadIdx.x, row = idx >> 4, c4 = idx & 15;
    if (PAIRS) {
      T* p = lds + row * QLD + 2 * c4;
      p[0] = pre[e][0];
      p[1] = pre[e][1];
      p[32] = pre[e][2];
      p[33] = pre[e][3];
    } else {
      *(t4*)(lds + row * QLD + 4 * c4) = pre[e];
    }
  }
}

// As tile_fetch for a matrix with nrows x ncols valid entries: zeros outside
// (16-byte reads where four columns are valid and aligned, else per element).
template <typename T>
__device__ inline void tile_fetch_guarded(const T* __restrict__ A, long ld, long r0, long c0,
                                          long nrows, long ncols, typename V4<T>::type (&pre)[4]) {
  typedef typename V4<T>::type t4;
  if (r0 + QT <= nrows && c0 + QT <= ncols && (ld & 3) == 0) {  // whole tile inside
    tile_fetch<T>(A, ld, r0, c0, pre);
    return;
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int idx = e * 256 + threadIdx.x, row = idx >> 4, c4 = idx & 15;
    const long r = r0 + row, c = c0 + 4 * c4;
    t4 v = {0, 0, 0, 0};
    if (r < nrows) {
      if ((ld & 3) == 0 && c + 3 < ncols) {
        v = *(const t4*)(A + r * ld + c);
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (c + j < ncols) v[j] = A[r * ld + c + j];
      }
    }
    pre[e] = v;
  }
}

// A fragments of 16 walkers (rows) over one k tile: a[4 u + j] holds
// ts[w][k0 + 16 u + 4 q + j] of walker w = w0 + li.  Rows beyond W read the
// last walker's row (no masked loads); the kernels never store those rows.
template <typename T>
__device__ inline void afrag_fetch(const T* __restrict__ ts, long Ktot, int W, int w0, long k0,
                                   int li, int q, T (&a)[16]) {
  typedef typename V4<T>::type t4;
  const int w = min(w0 + li, W - 1);
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const t4 v = *(const t4*)(ts + (long)w * Ktot + k0 + 16 * u + 4 * q);
#pragma unroll
    for (int j = 0; j < 4; ++j) a[4 * u + j] = v[j];
  }
}

// z[g][jb] += A_g (16 walkers x 64 k) times the LDS tile's columns 4 li + jb.
template <typename T, int GW>
__device__ inline void tile_mma(const T* lds, int li, int q, const T (&ar)[GW][16],
                                const T (&ai)[GW][16], typename Mfma<T>::acc_t (&zr)[GW][4],
                                typename Mfma<T>::acc_t (&zi)[GW][4]) {
  typedef typename V4<T>::type t4;
  typedef Mfma<T> MM;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const t4 b = *(const t4*)(lds + (16 * u + 4 * q + j) * QLD + 4 * li);
#pragma unroll
      for (int g = 0; g < GW; ++g)
#pragma unroll
        for (int jb = 0; jb < 4; ++jb) {
          zr[g][jb] = MM::mma(ar[g][4 * u + j], b[jb], zr[g][jb]);
          zi[g][jb] = MM::mma(ai[g][4 * u + j], b[jb], zi[g][jb]);
        }
    }
}

// As tile_mma for the NJ column tiles jb0 .. jb0 + NJ - 1 only.
template <typename T, int GW, int NJ>
__device__ inline void tile_mma_cols(const T* lds, int jb0, int li, int q, const T (&ar)[GW][16],
                                     const T (&ai)[GW][16], typename Mfma<T>::acc_t (&zr)[GW][NJ],
                                     typename Mfma<T>::acc_t (&zi)[GW][NJ]) {
  typedef Mfma<T> MM;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      // NJ == 2: the tile was stored with tile_store<T, true> (column pairs)
      T b[NJ];
      const int base = (16 * u + 4 * q + j) * QLD + (NJ == 2 ? (jb0 >> 1) * 32 + 2 * li : 4 * li + jb0);
#pragma unroll
      for (int jj = 0; jj < NJ; ++jj) b[jj] = lds[base + jj];
#pragma unroll
      for (int g = 0; g < GW; ++g)
#pragma unroll
        for (int jj = 0; jj < NJ; ++jj) {
          zr[g][jj] = MM::mma(ar[g][4 * u + j], b[jj], zr[g][jj]);
          zi[g][jj] = MM::mma(ai[g][4 * u + j], b[jj], zi[g][jj]);
        }
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Force-bias operand in the split order: Lq[soff_s + m N_s + a][g] =
// Ltil_g[a][m] of spin s (= Lt_s[g][m][a]), [Ktot][Gp], zero padded.
// ---------------------------------------------------------------------------
__global__ void k_build_lsplit(long n, int Gp, int G, int Kp0, int M, int MP4, int n_up, int n_dn,
                               int NP0, int NP1, const double* __restrict__ Lt0,
                               const double* __restrict__ Lt1, double* __restrict__ Lq) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const int k = (int)(e / Gp), g = (int)(e % Gp);
    const bool dn = k >= Kp0;
    const int kk = dn ? k - Kp0 : k, N = dn ? n_dn : n_up;
    double v = 0.0;
    if (g < G && kk < M * N) {
      const int m = kk / N, a = kk % N;
      v = dn ? Lt1[((long)g * MP4 + m) * NP1 + a] : Lt0[((long)g * MP4 + m) * NP0 + a];
    }
    Lq[e] = v;
  }
}

hipError_t build_lsplit(hipStream_t st, int G, int Gp, int M, int MP4, int n_up, int n_dn, int NP0,
                        int NP1, int Kp0, int Kp1, const double* Lt0, const double* Lt1,
                        double* Lq) {
  const long n = (long)(Kp0 + Kp1) * Gp;
  if (n == 0) return hipSuccess;
  const int blocks = (int)std::min<long>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_build_lsplit, dim3(blocks), dim3(256), 0, st, n, Gp, G, Kp0, M, MP4, n_up,
                     n_dn, NP0, NP1, Lt0, Lt1, Lq);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Q of one spin, [Kp][Kp] zero padded, from P = R^T R over the padded index
// (m NP + a) (R[g][m NP + a] = Lt[g][m][a]): Q[(n a)][(m b)] = P[(m a)][(n b)].
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_perm_qpad(long Kp, int K, int N, int NP, long LDP, const double* __restrict__ P,
                            T* __restrict__ Q) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < Kp * Kp; e += (long)gridDim.x * blockDim.x) {
    const long r = e / Kp, c = e % Kp;
    T v = 0;
    if (r < K && c < K) {
      const int nn = (int)(r / N), a = (int)(r % N), m = (int)(c / N), b = (int)(c % N);
      v = (T)P[((long)m * NP + a) * LDP + (long)nn * NP + b];
    }
    Q[e] = v;
  }
}

template <typename T>
hipError_t perm_qpad(hipStream_t st, int M, int N, int NP, int MP4, int Kp, const double* P, T* Q) {
  if (Kp == 0) return hipSuccess;
  const long n = (long)Kp * Kp;
  const int blocks = (int)std::min<long>((n + 255) / 256, 65536);
  hipLaunchKernelGGL((k_perm_qpad<T>), dim3(blocks), dim3(256), 0, st, (long)Kp, M * N, N, NP,
                     (long)MP4 * NP, P, Q);
  return hipGetLastError();
}
template hipError_t perm_qpad<double>(hipStream_t, int, int, int, int, int, const double*, double*);
template hipError_t perm_qpad<float>(hipStream_t, int, int, int, int, int, const double*, float*);

// ---------------------------------------------------------------------------
// Force bias v[w][g] = sum_k ts[w][k] Lq[k][g] (re and im rows of Theta as
// two A operands against one B), split over k into nz ranges of whole tiles:
// part[z][w][g].  Block = 4 waves x 16 walkers x 64 columns (one walker group
// per wave: two blocks per CU keep two waves per SIMD in flight); block index
// chunk-fastest, so with a multiple of 8 walker chunks each XCD keeps its
// chunks' Theta rows in its own L2.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_fbias_mm(int W, int Ktot, int G, int Gp, int nchunk,
                                                  int tiles_per_z, const T* __restrict__ tsr,
                                                  const T* __restrict__ tsi, const T* __restrict__ Lq,
                                                  T* __restrict__ part_re,
                                                  T* __restrict__ part_im) {
  constexpr int GW = 1;  // walker groups of 16 per wave
  typedef typename V4<T>::type t4;
  typedef Mfma<T> MM;
  __shared__ __attribute__((aligned(32))) T lds[2][QT * QLD];
  const int chunk = blockIdx.x % nchunk, rest = blockIdx.x / nchunk;
  const int ngt = Gp / QT, gt = rest % ngt, z = rest / ngt;
  const int nkt = Ktot / QT;
  const int kt0 = z * tiles_per_z, kt1 = min(nkt, kt0 + tiles_per_z);
  const int l = lane_id(), li = l & 15, q = l >> 4;
  const int wb = chunk * 64 * GW + wave_id() * 16 * GW;

  typename MM::acc_t zr[GW][4], zi[GW][4];
#pragma unroll
  for (int g = 0; g < GW; ++g)
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) zr[g][jb] = zi[g][jb] = MM::zero();
  T ar[GW][16], ai[GW][16];
  t4 pre[4];
  if (kt0 < kt1) {  // an empty range (k tiles fewer than ranges) writes zeros
    tile_fetch<T>(Lq, Gp, (long)kt0 * QT, (long)gt * QT, pre);
    tile_store<T, false>(lds[0], pre);
#pragma unroll
    for (int g = 0; g < GW; ++g) {
      afrag_fetch<T>(tsr, Ktot, W, wb + 16 * g, (long)kt0 * QT, li, q, ar[g]);
      afrag_fetch<T>(tsi, Ktot, W, wb + 16 * g, (long)kt0 * QT, li, q, ai[g]);
    }
  }
  __syncthreads();
  for (int kt = kt0; kt < kt1; ++kt) {
    const int buf = (kt - kt0) & 1;
    const bool more = kt + 1 < kt1;
    if (more) tile_fetch<T>(Lq, Gp, (long)(kt + 1) * QT, (long)gt * QT, pre);
    tile_mma<T, GW>(lds[buf], li, q, ar, ai, zr, zi);
    if (more) {
      tile_store<T, false>(lds[buf ^ 1], pre);
#pragma unroll
      for (int g = 0; g < GW; ++g) {
        afrag_fetch<T>(tsr, Ktot, W, wb + 16 * g, (long)(kt + 1) * QT, li, q, ar[g]);
        afrag_fetch<T>(tsi, Ktot, W, wb + 16 * g, (long)(kt + 1) * QT, li, q, ai[g]);
      }
    }
    __syncthreads();
  }
  const long zo = (long)z * W * G;
#pragma unroll
  for (int g = 0; g < GW; ++g)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int w = wb + 16 * g + MM::row(q, v);
      if (w >= W) continue;
#pragma unroll
      for (int jb = 0; jb < 4; ++jb) {
        const int c = gt * QT + 4 * li + jb;
        if (c < G) {
          part_re[zo + (long)w * G + c] = (T)zr[g][jb][v];
          part_im[zo + (long)w * G + c] = (T)zi[g][jb][v];
        }
      }
    }
}

int fbias_nz(int W, int Ktot, int G, long cap_per_walker) {
  const int nchunk = (W + 63) / 64;
  const int ngt = (G + QT - 1) / QT;
  const int nkt = Ktot / QT;
  // about 512 blocks (two per CU), within the partials' capacity
  int nz = std::max(1, std::min(nkt, (512 + nchunk * ngt - 1) / (nchunk * ngt)));
  return (int)std::max<long>(1, std::min<long>(nz, cap_per_walker / std::max(G, 1)));
}

template <typename T>
hipError_t fbias_mm(hipStream_t st, int W, int Ktot, int G, int Gp, int nz, const T* tsr,
                    const T* tsi, const T* Lq, T* part_re, T* part_im) {
  constexpr int GW = 1;
  const int nkt = Ktot / QT;
  if (W <= 0 || G <= 0 || nkt == 0 || nz < 1 || Gp % QT || Ktot % QT) return hipErrorInvalidValue;
  const int nchunk = (W + 64 * GW - 1) / (64 * GW);
  const int tpz = (nkt + nz - 1) / nz;
  const long blocks = (long)nchunk * (Gp / QT) * nz;
  hipLaunchKernelGGL((k_fbias_mm<T>), dim3((unsigned)blocks), dim3(256), 0, st, W, Ktot, G, Gp,
                     nchunk, tpz, tsr, tsi, Lq, part_re, part_im);
  return hipGetLastError();
}
template hipError_t fbias_mm<float>(hipStream_t, int, int, int, int, int, const float*,
                                    const float*, const float*, float*, float*);
template hipError_t fbias_mm<double>(hipStream_t, int, int, int, int, int, const double*,
                                     const double*, const double*, double*, double*);

// ---------------------------------------------------------------------------
// Propagator build (Eq. 2-3): A_prop[r][n] = sum_g coef[r][g] L[g][n] for the
// 2W rows r = 2 w + (re, im) of the shifted field coefficients (row-major,
// zero padded to Gp) and n over the M^2 operator entries; MFMA in TC, output
// rounded to TO.  Block = 4 waves x GW groups of 16 rows x 64 columns, row
// chunk fastest.
// ---------------------------------------------------------------------------
template <typename TC, typename TO>
__global__ __launch_bounds__(256) void k_abuild(int R, int Ncol, int G, int Gp, int nchunk,
                                                const TC* __restrict__ coef,
                                                const TC* __restrict__ L, TO* __restrict__ out) {
  constexpr int GW = QGeom<TC>::GW;
  typedef typename V4<TC>::type t4;
  typedef Mfma<TC> MM;
  __shared__ __attribute__((aligned(32))) TC lds[2][QT * QLD];
  const int chunk = blockIdx.x % nchunk, nt = blockIdx.x / nchunk;
  const int l = lane_id(), li = l & 15, q = l >> 4;
  const int rb = chunk * 64 * GW + wave_id() * 16 * GW;
  const int nkt = Gp / QT;
  typename MM::acc_t z[GW][4];
#pragma unroll
  for (int g = 0; g < GW; ++g)
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) z[g][jb] = MM::zero();
  TC ar[GW][16];
  t4 pre[4];
  tile_fetch_guarded<TC>(L, Ncol, 0, (long)nt * QT, G, Ncol, pre);
  tile_store<TC, false>(lds[0], pre);
#pragma unroll
  for (int g = 0; g < GW; ++g) afrag_fetch<TC>(coef, Gp, R, rb + 16 * g, 0, li, q, ar[g]);
  __syncthreads();
  for (int kt = 0; kt < nkt; ++kt) {
    const int buf = kt & 1;
    const bool more = kt + 1 < nkt;
    if (more) tile_fetch_guarded<TC>(L, Ncol, (long)(kt + 1) * QT, (long)nt * QT, G, Ncol, pre);
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const t4 b = *(const t4*)(lds[buf] + (16 * u + 4 * q + j) * QLD + 4 * li);
#pragma unroll
        for (int g = 0; g < GW; ++g)
#pragma unroll
          for (int jb = 0; jb < 4; ++jb) z[g][jb] = MM::mma(ar[g][4 * u + j], b[jb], z[g][jb]);
      }
    if (more) {
      tile_store<TC, false>(lds[buf ^ 1], pre);
#pragma unroll
      for (int g = 0; g < GW; ++g)
        afrag_fetch<TC>(coef, Gp, R, rb + 16 * g, (long)(kt + 1) * QT, li, q, ar[g]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int g = 0; g < GW; ++g)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const long r = rb + 16 * g + MM::row(q, v);
      if (r >= R) continue;
#pragma unroll
      for (int jb = 0; jb < 4; ++jb) {
        const long c = (long)nt * QT + 4 * li + jb;
        if (c < Ncol) out[r * Ncol + c] = (TO)z[g][jb][v];
      }
    }
}

template <typename TC, typename TO>
hipError_t abuild(hipStream_t st, int R, int Ncol, int G, int Gp, const TC* coef, const TC* L,
                  TO* out) {
  constexpr int GW = QGeom<TC>::GW;
  if (R <= 0 || Ncol <= 0 || G <= 0 || Gp % QT || Gp < G) return hipErrorInvalidValue;
  const int nchunk = (R + 64 * GW - 1) / (64 * GW);
  const long blocks = (long)nchunk * ((Ncol + QT - 1) / QT);
  hipLaunchKernelGGL((k_abuild<TC, TO>), dim3((unsigned)blocks), dim3(256), 0, st, R, Ncol, G, Gp,
                     nchunk, coef, L, out);
  return hipGetLastError();
}
template hipError_t abuild<float, float>(hipStream_t, int, int, int, int, const float*, const float*,
                                         float*);
template hipError_t abuild<float, double>(hipStream_t, int, int, int, int, const float*,
                                          const float*, double*);
template hipError_t abuild<double, float>(hipStream_t, int, int, int, int, const double*,
                                          const double*, float*);
template hipError_t abuild<double, double>(hipStream_t, int, int, int, int, const double*,
                                           const double*, double*);

// ---------------------------------------------------------------------------
// Quadratic form: segment (s, I, J0, J1) of spin s adds, for every walker of
// the block's chunk, f sum_{k in I, l in J} theta_k Q[k][l] theta_l over
// J0 <= J < J1 (f = 1 on the diagonal tile, 2 above it), into part[w][seg]
// (re, im).  theta_I stays in registers as the A operand; the Q tiles of the
// segment stream through double-buffered LDS; Z = theta_I Q_IJ is dotted
// with theta_J in the epilogue, per lane in FP64, and the 16 column lanes
// are summed once at the end in a fixed order.
// ---------------------------------------------------------------------------
// One group of 16 walkers per wavefront and all four column tiles in one
// pass; for FP32 the epilogue's theta_J values are requested before the
// tile's MFMAs, so that their latency hides behind them.
template <typename T> struct QFGeom {
  static constexpr int GW = 1, NJ = 4;
  static constexpr bool PREF = sizeof(T) == 4;
  static constexpr int WAVES = sizeof(T) == 4 ? 3 : 2;  // waves per SIMD (launch bound)
};

template <typename T>
__global__ __launch_bounds__(256, QFGeom<T>::WAVES) void k_qform(int W, int Ktot, int Kp0, int Kp1, int nchunk,
                                               int nseg, const int4* __restrict__ segs,
                                               const T* __restrict__ tsr, const T* __restrict__ tsi,
                                               const T* __restrict__ Q0, const T* __restrict__ Q1,
                                               double* __restrict__ part) {
  constexpr int GW = QFGeom<T>::GW, NJ = QFGeom<T>::NJ;
  constexpr bool PREF = QFGeom<T>::PREF;
  typedef typename V4<T>::type t4;
  typedef Mfma<T> MM;
  __shared__ __attribute__((aligned(32))) T lds[2][QT * QLD];
  const int chunk = blockIdx.x % nchunk, sg = blockIdx.x / nchunk;
  const int4 seg = segs[sg];
  const int s = seg.x, I0 = seg.y * QT;
  const long Kp = s ? Kp1 : Kp0;
  const long soff = s ? Kp0 : 0;
  const T* __restrict__ Q = s ? Q1 : Q0;
  const int l = lane_id(), li = l & 15, q = l >> 4;
  const int wb = chunk * 64 * GW + wave_id() * 16 * GW;

  T ar[GW][16], ai[GW][16];
#pragma unroll
  for (int g = 0; g < GW; ++g) {
    afrag_fetch<T>(tsr, Ktot, W, wb + 16 * g, soff + I0, li, q, ar[g]);
    afrag_fetch<T>(tsi, Ktot, W, wb + 16 * g, soff + I0, li, q, ai[g]);
  }
  double pr[GW][4], pim[GW][4];
#pragma unroll
  for (int g = 0; g < GW; ++g)
#pragma unroll
    for (int v = 0; v < 4; ++v) pr[g][v] = pim[g][v] = 0.0;

  t4 pre[4];
  tile_fetch<T>(Q, Kp, I0, (long)seg.z * QT, pre);
  tile_store<T, NJ == 2>(lds[0], pre);
  __syncthreads();
  for (int J = seg.z; J < seg.w; ++J) {
    const int buf = (J - seg.z) & 1;
    const bool more = J + 1 < seg.w;
    if (more) tile_fetch<T>(Q, Kp, I0, (long)(J + 1) * QT, pre);
    const double f = J == seg.y ? 1.0 : 2.0;
    t4 xpr[GW][4], xpi[GW][4];  // theta_J of the lane's rows (PREF)
    if (PREF) {
#pragma unroll
      for (int g = 0; g < GW; ++g)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int w = min(wb + 16 * g + MM::row(q, v), W - 1);
          const long o = (long)w * Ktot + soff + (long)J * QT + 4 * li;
          xpr[g][v] = *(const t4*)(tsr + o);
          xpi[g][v] = *(const t4*)(tsi + o);
        }
    }
#pragma unroll
    for (int jb0 = 0; jb0 < 4; jb0 += NJ) {
      typename MM::acc_t zr[GW][NJ], zi[GW][NJ];
#pragma unroll
      for (int g = 0; g < GW; ++g)
#pragma unroll
        for (int jj = 0; jj < NJ; ++jj) zr[g][jj] = zi[g][jj] = MM::zero();
      tile_mma_cols<T, GW, NJ>(lds[buf], jb0, li, q, ar, ai, zr, zi);
#pragma unroll
      for (int g = 0; g < GW; ++g)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          // rows beyond W repeat the last walker (afrag_fetch) and are not
          // stored; without the prefetch they are skipped (fewer live loads)
          const int wr = wb + 16 * g + MM::row(q, v);
          if (!PREF && wr >= W) continue;
          const int w = min(wr, W - 1);
          const long o = (long)w * Ktot + soff + (long)J * QT + 4 * li + jb0;
          double a = 0.0, b = 0.0;
#pragma unroll
          for (int jj = 0; jj < NJ; ++jj) {
            const double xr = PREF ? (double)xpr[g][v][jb0 + jj] : (double)tsr[o + jj];
            const double xi = PREF ? (double)xpi[g][v][jb0 + jj] : (double)tsi[o + jj];
            const double yr = (double)zr[g][jj][v], yi = (double)zi[g][jj][v];
            a += xr * yr - xi * yi;
            b += xr * yi + xi * yr;
          }
          pr[g][v] += f * a;
          pim[g][v] += f * b;
        }
    }
    if (more) tile_store<T, NJ == 2>(lds[buf ^ 1], pre);
    __syncthreads();
  }
#pragma unroll
  for (int g = 0; g < GW; ++g)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
#pragma unroll
      for (int o = 8; o >= 1; o >>= 1) {
        pr[g][v] += __shfl_xor(pr[g][v], o, AFQ_WAVE);
        pim[g][v] += __shfl_xor(pim[g][v], o, AFQ_WAVE);
      }
      const int w = wb + 16 * g + MM::row(q, v);
      if (li == 0 && w < W) {
        part[((long)w * nseg + sg) * 2] = pr[g][v];
        part[((long)w * nseg + sg) * 2 + 1] = pim[g][v];
      }
    }
}

template <typename T>
hipError_t qform(hipStream_t st, int W, int Kp0, int Kp1, int nseg, const int4* segs, const T* tsr,
                 const T* tsi, const T* Q0, const T* Q1, double* part) {
  constexpr int GW = QFGeom<T>::GW;
  if (nseg == 0) return hipSuccess;
  if (W <= 0 || Kp0 % QT || Kp1 % QT) return hipErrorInvalidValue;
  const int nchunk = (W + 64 * GW - 1) / (64 * GW);
  const long blocks = (long)nchunk * nseg;
  hipLaunchKernelGGL((k_qform<T>), dim3((unsigned)blocks), dim3(256), 0, st, W, Kp0 + Kp1, Kp0, Kp1,
                     nchunk, nseg, segs, tsr, tsi, Q0, Q1, part);
  return hipGetLastError();
}
template hipError_t qform<float>(hipStream_t, int, int, int, int, const int4*, const float*,
                                 const float*, const float*, const float*, double*);
template hipError_t qform<double>(hipStream_t, int, int, int, int, const int4*, const double*,
                                  const double*, const double*, const double*, double*);

// Q-route combination, one block of four waves per walker (many loads in
// flight per walker: the kernel only moves data): v_g = sum_z fpart[z][w][g]
// (the force-bias partials, fixed order), the exchange terms exx_s = sum over
// spin s's segments of qpart[w][seg], then E_L = e_core + E1 + 1/2 sum_g v_g^2
// - 1/2 (exx_0 + exx_1) and log S = log det_0 + log det_1 (Sec. II local
// energy); vfin = 0 when a force-bias entry is not finite.  The sums over
// threads are wave sums, then the four waves' values in wave order.
template <typename TP>
__global__ __launch_bounds__(256) void k_combine_qroute(
    int W, int G, int nz, int nseg0, int nseg1, double e_core, const TP* __restrict__ fp_re,
    const TP* __restrict__ fp_im, const double* __restrict__ qpart,
    const double* __restrict__ e1_re, const double* __restrict__ e1_im,
    const double* __restrict__ ld_re, const double* __restrict__ ld_im, double* __restrict__ v_re,
    double* __restrict__ v_im, double* exx_re, double* exx_im, double* lsn_re, double* lsn_im,
    double* eln_re, double* eln_im, int* vfin) {
  __shared__ double red[4][7];
  const int w = blockIdx.x, t = threadIdx.x, wv = wave_id(), l = lane_id();
  const long n = (long)W * G;
  double jr = 0.0, ji = 0.0, nonfin = 0.0;
  for (int g = t; g < G; g += blockDim.x) {
    double a = 0.0, b = 0.0;
    for (int z = 0; z < nz; ++z) {
      a += (double)fp_re[z * n + (long)w * G + g];
      b += (double)fp_im[z * n + (long)w * G + g];
    }
    v_re[(long)w * G + g] = a;
    v_im[(long)w * G + g] = b;
    jr += a * a - b * b;
    ji += 2.0 * a * b;
    if (!isfinite(a) || !isfinite(b)) nonfin = 1.0;
  }
  const int nseg = nseg0 + nseg1;
  const double* p = qpart + (long)w * nseg * 2;
  double x[2][2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int lo = s ? nseg0 : 0, hi = s ? nseg : nseg0;
    double a = 0.0, b = 0.0;
    for (int sg = lo + t; sg < hi; sg += blockDim.x) {
      a += p[2 * sg];
      b += p[2 * sg + 1];
    }
    x[s][0] = a;
    x[s][1] = b;
  }
  double v7[7] = {jr, ji, nonfin, x[0][0], x[0][1], x[1][0], x[1][1]};
#pragma unroll
  for (int k = 0; k < 7; ++k) v7[k] = wave_sum(v7[k]);
  if (l == 0) {
#pragma unroll
    for (int k = 0; k < 7; ++k) red[wv][k] = v7[k];
  }
  __syncthreads();
  if (t == 0) {
    double r[7];
#pragma unroll
    for (int k = 0; k < 7; ++k) r[k] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
    exx_re[2 * w] = r[3];
    exx_re[2 * w + 1] = r[5];
    exx_im[2 * w] = r[4];
    exx_im[2 * w + 1] = r[6];
    eln_re[w] = e_core + (e1_re[2 * w] + e1_re[2 * w + 1]) + 0.5 * r[0] - 0.5 * (r[3] + r[5]);
    eln_im[w] = (e1_im[2 * w] + e1_im[2 * w + 1]) + 0.5 * r[1] - 0.5 * (r[4] + r[6]);
    lsn_re[w] = ld_re[2 * w] + ld_re[2 * w + 1];
    lsn_im[w] = ld_im[2 * w] + ld_im[2 * w + 1];
    vfin[w] = r[2] == 0.0 ? 1 : 0;
  }
}

template <typename TP>
hipError_t combine_qroute(hipStream_t st, int W, int G, int nz, int nseg0, int nseg1, double e_core,
                          const TP* fp_re, const TP* fp_im, const double* qpart,
                          const double* e1_re, const double* e1_im, const double* ld_re,
                          const double* ld_im, double* v_re, double* v_im, double* exx_re,
                          double* exx_im, double* lsn_re, double* lsn_im, double* eln_re,
                          double* eln_im, int* vfin) {
  hipLaunchKernelGGL((k_combine_qroute<TP>), dim3(W), dim3(256), 0, st, W, G, nz, nseg0, nseg1,
                     e_core, fp_re, fp_im, qpart, e1_re, e1_im, ld_re, ld_im, v_re, v_im, exx_re,
                     exx_im, lsn_re, lsn_im, eln_re, eln_im, vfin);
  return hipGetLastError();
}
template hipError_t combine_qroute<float>(hipStream_t, int, int, int, int, int, double,
                                          const float*, const float*, const double*, const double*,
                                          const double*, const double*, const double*, double*,
                                          double*, double*, double*, double*, double*, double*,
                                          double*, int*);
template hipError_t combine_qroute<double>(hipStream_t, int, int, int, int, int, double,
                                           const double*, const double*, const double*,
                                           const double*, const double*, const double*,
                                           const double*, double*, double*, double*, double*,
                                           double*, double*, double*, double*, int*);

}  // namespace afq
