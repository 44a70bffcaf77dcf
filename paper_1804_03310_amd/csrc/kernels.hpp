// Launchers of the gfx950 kernels (host side).  Every launcher enqueues on
// `st` and returns the hipError_t of the launch.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace afq {

// Per-spin parameters of one system, shared by several kernels.
struct SpinGeom {
  int N;              // electrons of this spin
  int off;            // first column of this spin in a walker matrix
  int NP;             // N rounded up to a multiple of 16
  const double* C;    // [M][M] orbitals, D_0 = columns 0..N-1
  const double* htil; // [N][M] = D_0^T h
  const void* Lt;     // [G][MP4][NP] half-rotated Cholesky, D_0^T L_g, transposed, zero padded
  const void* Apk;    // Lt repacked as the exchange kernels' A operand, KB = ceil(MP4 / 16):
                      // NP <= 32: [G][KB][64 lanes][4 k steps][NP / 16] (FP64 and FP32);
                      // 32 < NP <= 64: [G][NP / 16][KB][64 lanes][4 k steps] (FP32)
};

// C[z] = alpha * A[z] B[z]; A(m,k) = A_KMAJ ? A[k*lda+m] : A[m*lda+k], B(k,n) = B[k*ldb+n].
template <typename TIn, typename TOut, bool A_KMAJ>
hipError_t gemm_real(hipStream_t st, int Mr, int Nc, int K, const TIn* A, int lda, long sA,
                     const TIn* B, int ldb, long sB, TOut* C, int ldc, long sC, int batch,
                     double alpha);

// Walker-batched complex product of an M x K operator with K x Nc walker columns.
// mode 0: D1 = In + A In (and D2 = D1 if D2 != null); A real, shared.
// mode 1: Out = alpha A In (type T), D1 += alpha A In; A complex per walker.
template <typename T, typename TIn, bool A_CPLX, int MODE>
hipError_t cgemm_walkers(hipStream_t st, int W, int Mr, int Nc, int K, const T* Ar, const T* Ai,
                         int lda, long sA, const TIn* Inr, const TIn* Ini, int ldin, long sIn,
                         T* Outr, T* Outi, double* D1r, double* D1i, double* D2r, double* D2i,
                         int ldo, long sO, double alpha);

// Fields x, shifted propagator coefficients coef[2w + {0,1}][g] = i sqrt(dt)(x - xbar)
// (re, im rows of length ldc >= G, zeros beyond G) and the mean-field log factor mf[w].
template <typename T>
hipError_t fields_coeff(hipStream_t st, int W, int G, int ldc, uint64_t seed, uint64_t t,
                        int system_id, double dt, const double* v_re, const double* v_im,
                        const double* lbar, T* coef, double* mf_re, double* mf_im, double* xdump,
                        double* hy_re = nullptr, double* hy_im = nullptr);

// Where the overlap kernels put Theta: the FP64 matrix th[w][m][Nt] (thr
// non-null) and/or the split rows of the Q route ts[w][Ktot] (sr non-null;
// float when f32, else double), spin 0's (m b) at m N_up + b, spin 1's from
// Kp0, the padding up to each spin's 64-multiple written as zeros.
struct ThetaOut {
  double* thr = nullptr;
  double* thi = nullptr;
  void* sr = nullptr;
  void* si = nullptr;
  int Ktot = 0, Kp0 = 0;
  bool f32 = true;
};

// Per (walker, spin): S = D_0^T phi, LU/Gauss-Jordan inverse, log det, Theta = phi S^-1,
// E1 = Tr(htil Theta).
hipError_t overlap_theta(hipStream_t st, int W, int M, int Nt, SpinGeom s0, SpinGeom s1,
                         const double* phr, const double* phi, ThetaOut to, double* ld_re,
                         double* ld_im, double* e1_re, double* e1_im, size_t max_lds);

// Per (walker, spin): X_g = Ltil_g Theta; v[w][s][g] = Tr X_g; exx[w][s] = sum_g Tr(X_g X_g).
// Repack Lt [G][MP4][NP] (NP = 16 NT) into the A-operand order of the
// exchange kernels: for slab g, batch kb of four k steps and lane
// l = li + 16 lk, the values Lt[g][4 (4 kb + j) + lk][16 I + li] (j < 4,
// I < NT) with j and I innermost for NP <= 32 and I outermost (after g) for
// 32 < NP <= 64; rows past MP4 are zero.
template <typename T>
hipError_t pack_exchange_a(hipStream_t st, int G, int MP4, int NP, const T* Lt, T* Apk);

template <typename T>
hipError_t exchange(hipStream_t st, int W, int M, int MP4, int Nt, int G, SpinGeom s0, SpinGeom s1,
                    const double* thr, const double* thi, double* vs_re, double* vs_im,
                    double* exx_re, double* exx_im, size_t max_lds);

// Per walker: v = v_up + v_dn, E_L, log S_new (single determinant).
hipError_t combine_single(hipStream_t st, int W, int G, double e_core, const double* vs_re,
                          const double* vs_im, const double* exx_re, const double* exx_im,
                          const double* e1_re, const double* e1_im, const double* ld_re,
                          const double* ld_im, double* v_re, double* v_im, double* lsn_re,
                          double* lsn_im, double* eln_re, double* eln_im, int* vfin);

// mode 0: logS, eloc <- new values.  mode 1: phaseless weight update in the local-energy
// form.  mode 2: logS only.  modes 3 / 4: hybrid form (hy = sum_g (x xbar - xbar^2/2),
// e0 = E_0) with / without taking the new E_L.
hipError_t weight_update(hipStream_t st, int W, int mode, double dt, double e_trial,
                         const double* lsn_re, const double* lsn_im, const double* eln_re,
                         const double* eln_im, const double* mf_re, const double* mf_im,
                         const int* vfin, double* weight, double* logS_re, double* logS_im,
                         double* eloc_re, double* eloc_im, int* dead,
                         const double* hy_re = nullptr, const double* hy_im = nullptr,
                         double e0 = 0.0);

// Dead walkers back to the reference determinant and its state.
hipError_t reset_dead(hipStream_t st, int W, int M, int Nt, int G, const int* dead,
                      const double* D0, double ref_ls_re, double ref_ls_im, double ref_el_re,
                      double ref_el_im, const double* vref_re, const double* vref_im,
                      double* phr, double* phi, double* logS_re, double* logS_im,
                      double* eloc_re, double* eloc_im, double* v_re, double* v_im);

// emix_out[0] = sum W Re E_L / sum W; den_out (nullable) = sum W.
hipError_t mixed_energy(hipStream_t st, int W, const double* weight, const double* eloc_re,
                        double* emix_out, double* den_out);

// Modified Gram-Schmidt of both spin blocks of every walker, in place.
hipError_t mgs(hipStream_t st, int W, int M, int Nt, int n_up, int n_dn, double* phr, double* phi,
               size_t max_lds);

// Comb: parents and norm factor (single thread, left-to-right sums).  With no
// positive finite total weight: identity parents and norm factor 0.
hipError_t comb_parents(hipStream_t st, int W, const double* weight, uint64_t seed,
                        uint64_t pc_index, int system_id, double* cbuf, int* parent,
                        double* norm_out);
// Weights after the comb: 1 where the norm factor is positive, else unchanged.
hipError_t comb_weights(hipStream_t st, int W, const double* norm, double* weight);
// Gather rows of length `row` doubles from src[parent[j]] to dst[j], for `nbuf` buffers.
hipError_t gather_rows(hipStream_t st, int W, long row, const int* parent, const double* src,
                       double* dst);
// The same gather through a snapshot of at most snap_doubles doubles
// (>= W): column ranges of the rows are snapshotted and gathered in turn,
// so src_dst is updated in place through a bounded buffer.
hipError_t gather_rows_chunked(hipStream_t st, int W, long row, const int* parent,
                               double* src_dst, double* snap, size_t snap_doubles);
hipError_t fill(hipStream_t st, double* p, long n, double value);
hipError_t broadcast_rows(hipStream_t st, int W, long row, const double* src, double* dst);

// lbar[g] += sum_{m,a} Lt[g][m][a] C[m][a]
hipError_t lbar_accumulate(hipStream_t st, int G, int M, int MP4, int N, int NP, const double* Lt,
                           const double* C, double* lbar);
hipError_t convert_f64_f32(hipStream_t st, const double* src, float* dst, long n);

}  // namespace afq

namespace afq {

// Multi-determinant trial (Sec. III).  Per spin: N, column offset, orbitals C
// [M][M] (FP64) and the rotated Cholesky tensor LC [G+1][M][M] in the
// contraction type, LC[g][m][p] = (L_g C)[m][p] and LC[G] = h C.
struct MDSpin {
  int N;
  int off;
  const double* C;
  const void* LC;
};
// Compact-row tables of the FP32 energy kernel.  Per spin only the rows of
// C^T O Theta_0 that some determinant reads are formed: the N occupied rows,
// then the distinct particle orbitals in ascending order (R rows, padded to
// RP, a multiple of 16).  A (particle, hole) pair whose sums over the occupied
// index a determinant needs is listed once per spin.
struct MDRows {
  int ok;                // the tables exist (M <= 128, N <= 16, at most 64 particles per
                         // spin, n_det <= 256)
  int KS;                // k steps of the operators: 16 (M <= 64) or 32
  int R[2], RP[2], npair[2];
  const float* LCc[2];   // [G+2][4 KS x RP, MFMA fragment order]: slot g <= G the rows of
                         // LC[g], slot G+1 the rows of C
  const int* pair[2];    // [npair]: (t << 8) | r, t the particle's compact index minus N,
                         // ordered by t then r
  const int* pbeg[2];    // [R - N + 1]: the pairs of particle t are pbeg[t] .. pbeg[t+1]-1
  const int* dx;         // [n_det][kMdDx]: per slot, three packed words per spin, then
                         // the determinant's index in the trial's list
};
// Packed per-(determinant, spin) words: w0 = E | r0 << 2 | r1 << 7 | t0 << 12 |
// t1 << 20; w1 = pair(0,0) | pair(0,1) << 16; w2 = pair(1,0) | pair(1,1) << 16.
constexpr int kMdDx = 7;
constexpr int kMdRowsMaxM = 128;
constexpr int kMdRowsMaxN = 16;
constexpr int kMdRowsMaxDet = 256;
constexpr int kMdRowsPF = 12;  // float4 staging registers per thread: 4 KS RP <= 12288
struct MDParams {
  int M, Nt, G, n_det, MP4;
  double e_core;
  MDSpin sp[2];
  const int* exc;        // [n_det][2][5] = (E, hole0, hole1, particle0, particle1)
  const double* coeff;   // [n_det]
  MDRows rows;
};

// LCc[slot] = (float) src[slot][m][rowmap[c]] (m < M, c < R; zero elsewhere in
// the 4 KS x RP block) in the energy kernel's MFMA fragment order.
hipError_t md_rows_gather(hipStream_t st, int nslot, int M, int KS, int R, int RP,
                          const int* rowmap, const double* src, float* dst);

// Per walker: Ghat = C^T Theta_0 (FP64), overlap ratio of every determinant
// c0[w][s][i] = det(Ghat[particles, holes]), the total relative overlap
// tot[w] = sum_i c_i c0_up c0_dn, and log S = sum_s log det A_s + log tot.
hipError_t md_overlap(hipStream_t st, int W, const MDParams& p, const double* thr,
                      const double* thi, const double* ld_re, const double* ld_im,
                      double* c0_re, double* c0_im, double* tot_re, double* tot_im,
                      double* lsn_re, double* lsn_im, size_t max_lds);

// Per walker: E_L, force-bias input v and finiteness flag for the
// multi-determinant trial, from the reference Theta_0 and the ratios above.
template <typename T>
hipError_t md_energy(hipStream_t st, int W, const MDParams& p, const double* thr,
                     const double* thi, const double* c0_re, const double* c0_im,
                     const double* tot_re, const double* tot_im, double* v_re, double* v_im,
                     double* eln_re, double* eln_im, int* vfin, size_t max_lds);

}  // namespace afq

namespace afq {
// BF16 contraction path (bf16.hip).
// Split bf16 operands (BF16X3): x = hi + lo, hi = bf16(x), lo = bf16(x - hi).
hipError_t convert_f64_bf16(hipStream_t st, const double* src, void* dst, long n);
hipError_t convert_f64_bf16_lo(hipStream_t st, const double* src, void* dst, long n);
// Ltil_g from its FP64 [G][MP4][NP] copy into the bf16 exchange kernels' fragment order,
// [G][NPX / 16][MP32 / 32][64 lanes] groups of eight (rows a >= NP and columns m >= MP4 zero);
// lo (nullable) receives the split's second terms.
hipError_t pack_ltilde_bf16(hipStream_t st, int G, int MP4, int NP, int NPX, int MP32,
                            const double* src, void* hi, void* lo);
// Al / Bl non-null: the three-product split form.
template <typename TOut>
hipError_t gemm_bf16(hipStream_t st, int Mr, int Nc, int K, const void* A, const void* Al, int lda,
                     const void* B, const void* Bl, int ldb, TOut* C, int ldc, double alpha);
// Hybrid weights: v from the force-bias GEMM's split-K partials summed here;
// lsn = ld_up + ld_dn and vfin = all v finite per walker.
template <typename TP>
hipError_t hybrid_force_bias_finish(hipStream_t st, int W, int G, int nz, const TP* part_re,
                                    const TP* part_im, double* v_re, double* v_im,
                                    const double* ld_re, const double* ld_im, double* lsn_re,
                                    double* lsn_im, int* vfin);
// Q route (qroute.hip), over the split Theta rows ts[w][Ktot] that the
// overlap kernels write (ThetaOut).
// Lq[k][g] ([Ktot][Gp], zero padded): Ltil_g[a][m] at the split index of (s, m, a).
hipError_t build_lsplit(hipStream_t st, int G, int Gp, int M, int MP4, int n_up, int n_dn, int NP0,
                        int NP1, int Kp0, int Kp1, const double* Lt0, const double* Lt1,
                        double* Lq);
// Q[(n a)][(m b)] = P[(m NP + a)][(n NP + b)] into [Kp][Kp], zero padded.
template <typename T>
hipError_t perm_qpad(hipStream_t st, int M, int N, int NP, int MP4, int Kp, const double* P, T* Q);
// Number of k ranges of the force-bias GEMM (about 512 blocks; partials of
// nz W G elements must fit cap_per_walker W doubles).
int fbias_nz(int W, int Ktot, int G, long cap_per_walker);
// part[z][w][g] = sum over range z of ts[w][k] Lq[k][g], re and im (in T: the
// partial sums as the MFMA accumulated them).
template <typename T>
hipError_t fbias_mm(hipStream_t st, int W, int Ktot, int G, int Gp, int nz, const T* tsr,
                    const T* tsi, const T* Lq, T* part_re, T* part_im);
// part[w][seg] (re, im) of theta^T Q theta over the segment's tile pairs.
template <typename T>
hipError_t qform(hipStream_t st, int W, int Kp0, int Kp1, int nseg, const int4* segs, const T* tsr,
                 const T* tsi, const T* Q0, const T* Q1, double* part);
// Propagator build out[r][n] = sum_g coef[r][g] L[g][n], coef [R][Gp] row-major
// (zero padded), L [G][Ncol]; MFMA in TC, output in TO.
template <typename TC, typename TO>
hipError_t abuild(hipStream_t st, int R, int Ncol, int G, int Gp, const TC* coef, const TC* L,
                  TO* out);
// Q-route E_L: force bias from nz partials, exchange from the segment partials,
// combined with E1 and log det (one wave per walker).
template <typename TP>
hipError_t combine_qroute(hipStream_t st, int W, int G, int nz, int nseg0, int nseg1, double e_core,
                          const TP* fp_re, const TP* fp_im, const double* qpart,
                          const double* e1_re, const double* e1_im, const double* ld_re,
                          const double* ld_im, double* v_re, double* v_im, double* exx_re,
                          double* exx_im, double* lsn_re, double* lsn_im, double* eln_re,
                          double* eln_im, int* vfin);
// coef_lo (nullable): the split's second terms of the coefficients.
hipError_t fields_coeff_bf16(hipStream_t st, int W, int G, int ldg, uint64_t seed, uint64_t t,
                             int system_id, double dt, const double* v_re, const double* v_im,
                             const double* lbar, void* coef, void* coef_lo, double* mf_re,
                             double* mf_im, double* hy_re = nullptr, double* hy_im = nullptr);
// Lt_lo0 / Lt_lo1 non-null: the three-product split form.
hipError_t exchange_bf16(hipStream_t st, int W, int M, int MP32, int Nt, int G, SpinGeom s0,
                         SpinGeom s1, const void* Lt_lo0, const void* Lt_lo1, const double* thr,
                         const double* thi, double* vs_re, double* vs_im, double* exx_re,
                         double* exx_im, size_t max_lds);
}  // namespace afq

namespace afq {
// Fused B1 exp(A) B1 for small M (one block per walker; see kernels.hip).
// packed: A per walker as the upper triangles [2][M (M + 1) / 2] (re, im)
// instead of [2][M][M].
template <typename T>
hipError_t propagate_fused(hipStream_t st, int W, int M, int Nt, int order, bool packed,
                           const T* A, const T* B1m, double* phr, double* phi, size_t max_lds);
bool propagate_fused_fits(int M, int Nt, size_t elem, size_t max_lds);
}  // namespace afq
