// Device helpers shared by the gfx950 kernels: MFMA tile wrappers, wave and
// block reductions, the Philox4x64-10 counter generator, complex scalars.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define AFQ_WAVE 64

typedef double afq_d4 __attribute__((ext_vector_type(4)));
typedef float afq_f4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// 16x16x4 MFMA tiles.  For both the f64 and the f32 instruction a lane l
// supplies A[i = l%16][k = l/16] and B[k = l/16][j = l%16].  Accumulator
// entry v = 0..3 of lane l holds D[row(l/16, v)][l%16], where
// row = 4*(l/16) + v for f32 and row = l/16 + 4*v for f64 (checked on gfx950
// hardware with an in-bounds probe).
// ---------------------------------------------------------------------------
template <typename T> struct Mfma;

template <> struct Mfma<double> {
  typedef afq_d4 acc_t;
  __device__ static inline acc_t zero() { return acc_t{0.0, 0.0, 0.0, 0.0}; }
  __device__ static inline acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lk, int v) { return lk + 4 * v; }
};

template <> struct Mfma<float> {
  typedef afq_f4 acc_t;
  __device__ static inline acc_t zero() { return acc_t{0.f, 0.f, 0.f, 0.f}; }
  __device__ static inline acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lk, int v) { return 4 * lk + v; }
};

__device__ inline int lane_id() { return threadIdx.x & (AFQ_WAVE - 1); }
// The wavefront's index in its block, marked wave-uniform (a scalar value), so
// that what depends on it only (branches, addresses) stays scalar.
__device__ inline int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x / AFQ_WAVE); }

// Intra-wave LDS hand-off: make this wave's LDS writes visible to its lanes.
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Butterfly sum over the 64 lanes of a wave; every lane gets the total.  The
// combination order is fixed, so results are bitwise reproducible.
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, AFQ_WAVE);
  return v;
}

__device__ inline float wave_sum_t(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, AFQ_WAVE);
  return v;
}
__device__ inline double wave_sum_t(double v) { return wave_sum(v); }

// Sum over the lanes {0..3, 20..23, 40..43, 60..63}, which hold the diagonal
// of a 16x16 f32 MFMA result tile (lane (li, lk) holds rows 4 lk .. 4 lk + 3
// of column li); returned in every lane.  Quad sums by DPP, then the four
// quads by lane reads, in a fixed order.
__device__ inline float quad_sum_dpp(float x) {
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0xB1, 0xF, 0xF, false));
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x4E, 0xF, 0xF, false));
  return x;
}
__device__ inline float diag16_sum(float x) {
  const int q = __float_as_int(quad_sum_dpp(x));
  const float a = __int_as_float(__builtin_amdgcn_readlane(q, 0));
  const float b = __int_as_float(__builtin_amdgcn_readlane(q, 20));
  const float c = __int_as_float(__builtin_amdgcn_readlane(q, 40));
  const float d = __int_as_float(__builtin_amdgcn_readlane(q, 60));
  return (a + b) + (c + d);
}

// Fixed-order block sum of one double per thread (blockDim.x <= 1024,
// a multiple of 64).  `red` is LDS scratch of blockDim.x/64 doubles.  All
// threads return the total.
__device__ inline double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int nw = blockDim.x / AFQ_WAVE;
  __syncthreads();
  if (lane_id() == 0) red[wave_id()] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < nw; ++i) t += red[i];
  __syncthreads();
  return t;
}

// ---------------------------------------------------------------------------
// Philox4x64 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11).
// ---------------------------------------------------------------------------
struct PhiloxOut { uint64_t w[4]; };

__device__ inline PhiloxOut philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                          uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += W0; k1 += W1; }
    const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
    const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  PhiloxOut o;
  o.w[0] = c0; o.w[1] = c1; o.w[2] = c2; o.w[3] = c3;
  return o;
}

// Top 53 bits to a double in (0,1).
__device__ inline double u64_to_unit(uint64_t r) {
  return ((double)(r >> 11) + 0.5) * 1.1102230246251565404236316680908203125e-16;
}

#define AFQ_STREAM_FIELDS 0ull
#define AFQ_STREAM_COMB 1ull

// Four standard normals for counter (t, walker, q, system): Box-Muller on
// (u0,u1) and (u2,u3); entry j belongs to field gamma = 4q + j.
__device__ inline void gaussian4(uint64_t seed, uint64_t t, uint64_t walker, uint64_t q,
                                 uint64_t system, double z[4]) {
  PhiloxOut r = philox4x64_10(t, walker, q, system, seed, AFQ_STREAM_FIELDS);
  const double u0 = u64_to_unit(r.w[0]), u1 = u64_to_unit(r.w[1]);
  const double u2 = u64_to_unit(r.w[2]), u3 = u64_to_unit(r.w[3]);
  const double r01 = sqrt(-2.0 * log(u0)), r23 = sqrt(-2.0 * log(u2));
  // cos and sin of 2 pi u with one reduction each (2 u is exact)
  double s1, c1, s3, c3;
  sincospi(2.0 * u1, &s1, &c1);
  sincospi(2.0 * u3, &s3, &c3);
  z[0] = r01 * c1;
  z[1] = r01 * s1;
  z[2] = r23 * c3;
  z[3] = r23 * s3;
}

// ---------------------------------------------------------------------------
// Complex scalars (double).
// ---------------------------------------------------------------------------
struct zdbl { double re, im; };
__device__ inline zdbl zmul(zdbl a, zdbl b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline zdbl zadd(zdbl a, zdbl b) { return {a.re + b.re, a.im + b.im}; }
__device__ inline zdbl zsub(zdbl a, zdbl b) { return {a.re - b.re, a.im - b.im}; }
__device__ inline zdbl zdiv(zdbl a, zdbl b) {
  // Smith's algorithm
  if (fabs(b.re) >= fabs(b.im)) {
    const double r = b.im / b.re, d = b.re + b.im * r;
    return {(a.re + a.im * r) / d, (a.im - a.re * r) / d};
  } else {
    const double r = b.re / b.im, d = b.re * r + b.im;
    return {(a.re * r + a.im) / d, (a.im * r - a.re) / d};
  }
}
__device__ inline zdbl zlog(zdbl a) { return {log(hypot(a.re, a.im)), atan2(a.im, a.re)}; }

template <typename T> __device__ inline T to_t(double x) { return (T)x; }

// ---------------------------------------------------------------------------
// BF16 16x16x32 MFMA (gfx950): lane l supplies A[i = l%16][k = 8*(l/16) + j]
// and B[k = 8*(l/16) + j][n = l%16] for j = 0..7 (eight bf16 each, packed in
// one 16-byte vector); accumulator entry v holds D[4*(l/16) + v][l%16] in FP32.
// ---------------------------------------------------------------------------
typedef __bf16 afq_bf8 __attribute__((ext_vector_type(8)));
__device__ inline afq_f4 mfma_bf16(afq_bf8 a, afq_bf8 b, afq_f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ inline int row_bf16(int lk, int v) { return 4 * lk + v; }
