// Walker-resident propagation of several systems in one launch: host/device
// shared description of a group member and of a walker block's LDS layout.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace afq {

// Largest systems the resident kernel takes: one wavefront owns the rows of a
// spin block in MGS (M <= 64) and the rows of an overlap matrix in the
// elimination (N <= 64); the walker's arrays and the staged operators must
// fit one CU's LDS (tiny systems: the latency-bound regime).
constexpr int kResMaxM = 64;
constexpr int kResMaxMembers = 64;

// One member (system) of a group, as the kernels read it from device memory.
struct ResMember {
  int M, Nt, n0, n1, G, W;
  int wbase;        // first walker block of this member in the launch
  int system_id;    // Philox counter word 3
  int ortho_every;  // 0: never
  int pc_every;     // 0: never
  int MP4, NP0, NP1;
  int order;        // Taylor order
  uint64_t seed;
  uint64_t call_step0;  // global step index of the first step of the current call
  double dt, sqdt, e_trial, e_core;
  double ref_ls_re, ref_ls_im, ref_el_re, ref_el_im;
  const double* L;     // [G][M][M]
  const double* B1m;   // [M][M], B1 - I
  const double* D0;    // [M][Nt]
  const double* Lt0;   // [G][MP4][NP0]: Ltil_g[a][m] at (g MP4 + m) NP0 + a
  const double* Lt1;
  const double* ht0;   // [n0][M]
  const double* ht1;
  const double* lbar;  // [G]
  const double* vref_re;
  const double* vref_im;
  double* phi_re;      // [W][M][Nt]
  double* phi_im;
  double* weight;
  double* ls_re;
  double* ls_im;
  double* el_re;
  double* el_im;
  double* v_re;        // [W][G]
  double* v_im;
  double* emix;        // [steps of the current call] or null
  // comb scratch
  double* snap;        // [W][2 M Nt + 4 + 2 G]
  int* parent;         // [W]
  double* cbuf;        // [W]
  double* comb_scal;   // [0] norm factor, [1] 1.0 if this member combed in the segment
};

// Offsets (in doubles) of a walker block's LDS arrays; the same function on
// the host (launch size) and the device (carving).
// The second part holds the member's operators, staged once per segment:
// B1 - I [M][M], D_0 [M][Nt], htil [Nt][M] (spin 0's rows, then spin 1's),
// lbar [G], Ltil [G][n0][M] then [G][n1][M], L [G][M][M].
// Xg holds X_g = Ltil_g Theta of one spin for every g ([G][Nx][Nx], Nx the
// larger spin count), pt / px the per-row partials of Tr X and Tr(X X).
struct ResLds {
  int ph_r, ph_i, A_r, A_i, X_r, X_i, Y_r, Y_i, Z_r, Z_i;
  int cf_r, cf_i, v_r, v_i, tr_r, tr_i, xx_r, xx_i, red, sc;
  int Xg_r, Xg_i, pt_r, pt_i, px_r, px_i;
  int B1, D0, ht, lb, Lt, L;
  int total;
};

__host__ __device__ inline ResLds res_lds(int M, int Nt, int G, int Nx) {
  ResLds o;
  const int mn = M * Nt, mm = M * M, G1 = G > 0 ? G : 1, nq = (G + 3) / 4;
  int p = 0;
  o.ph_r = p; p += mn;
  o.ph_i = p; p += mn;
  o.A_r = p; p += mm;
  o.A_i = p; p += mm;
  o.X_r = p; p += mn;
  o.X_i = p; p += mn;
  o.Y_r = p; p += mn;
  o.Y_i = p; p += mn;
  o.Z_r = p; p += mn;
  o.Z_i = p; p += mn;
  o.cf_r = p; p += G1;
  o.cf_i = p; p += G1;
  o.v_r = p; p += G1;
  o.v_i = p; p += G1;
  o.tr_r = p; p += 2 * G1;
  o.tr_i = p; p += 2 * G1;
  o.xx_r = p; p += 2 * G1;
  o.xx_i = p; p += 2 * G1;
  o.red = p; p += 2 * (nq > Nt ? nq : Nt);
  o.sc = p; p += 32;
  o.Xg_r = p; p += G1 * Nx * Nx;
  o.Xg_i = p; p += G1 * Nx * Nx;
  o.pt_r = p; p += G1 * Nx;
  o.pt_i = p; p += G1 * Nx;
  o.px_r = p; p += G1 * Nx;
  o.px_i = p; p += G1 * Nx;
  o.B1 = p; p += mm;
  o.D0 = p; p += mn;
  o.ht = p; p += mn;
  o.lb = p; p += G1;
  o.Lt = p; p += G * mn;
  o.L = p; p += G * mm;
  o.total = p;
  return o;
}

// Launchers (resident.hip).  `tdev` holds the global index of the segment's
// first step; every kernel of a segment reads it, and res_advance moves it on,
// so that one captured segment replays as the next.
hipError_t res_steps(hipStream_t st, const ResMember* mem, int n_mem, int w_total, int threads,
                     size_t lds_bytes, const uint64_t* tdev, int K, int refresh, double* wsum);
hipError_t res_emix(hipStream_t st, const ResMember* mem, int n_mem, int w_total,
                    const uint64_t* tdev, int K, const double* wsum);
hipError_t res_comb(hipStream_t st, const ResMember* mem, int n_mem, int w_total,
                    const uint64_t* tdev, int K, int w_max);
hipError_t res_advance(hipStream_t st, uint64_t* tdev, int K);
hipError_t res_begin(hipStream_t st, ResMember* mem, int n_mem, uint64_t* tdev, uint64_t step0,
                     double* const* emix);

}  // namespace afq
