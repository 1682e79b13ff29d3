// Internal declarations shared by the host runtime and the HIP kernels of the
// ADG library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace adg {

constexpr int kMaxM = 5;      // N_p <= 4
constexpr int kMaxQ = 5;      // Gauss points = N_p + 1
constexpr int kMaxL = 8;      // admissible delays
constexpr int kMaxAT = 6;     // AT order q
constexpr int kEulerBlock = 256;

// Delay model of Sec. 4 (CAA / SAA) and the start-up clamp k <= n - q + 1.
struct DelayParams {
  int mode;        // 0 sync, 1 CAA, 2 SAA, 3 schedule
  int L;
  int nif;
  int q;
  int sched_steps;
  double cum[kMaxL];            // cumulative SAA probabilities (summed left to right)
  unsigned long long seed;
  const int8_t *sched;          // device [sched_steps][nif]
  int hybrid;                   // buffer-element DoFs (Eq. (11)): mode j from max(1, q - j) levels
};

// History of past levels at PE interfaces: D slots (level n lives in slot n mod D),
// 3 stages, nif interfaces; one record per (slot, stage, interface) of `rec` doubles:
// [F: V][Wc: V][U_left: V*M][U_right: V*M]  (Wc only for LDG, U only with the limiter).
struct RingParams {
  double *base;
  int D;
  int stages;           // RK stages per time step (records per level)
  int rec;
  int off_F, off_Wc, off_U;
};

// Device state layout: blocks of 64 elements, each block holding its V*M
// component segments of 64 consecutive elements: [E/64][V*M][64].  A wavefront
// reading one component of 64 neighbouring elements issues one contiguous
// 512-byte access, and all components of those elements lie in one 64*V*M*8
// byte span.
constexpr int kLayoutBlock = 64;
__host__ __device__ inline size_t sidx(int e, int c, int VM) {
  return ((size_t)(e >> 6) * VM + c) * kLayoutBlock + (e & 63);
}
__host__ __device__ inline size_t state_doubles(int E, int VM) {
  return (size_t)((E + kLayoutBlock - 1) / kLayoutBlock) * kLayoutBlock * VM;
}

// Record of (slot, stage, interface i).  Level n - b (0 <= b < D) lives in slot
// ring_slot(n mod D, b): a kernel forms n mod D once and steps back from it.
__host__ __device__ inline int ring_slot(int n_mod_d, int back, int D) {
  const int s = n_mod_d - back;
  return s < 0 ? s + D : s;
}
__host__ __device__ inline double *ring_at(const RingParams &r, int slot, int stage, int nif, int i) {
  return r.base + ((size_t)(slot * r.stages + stage) * (size_t)nif + (size_t)i) * (size_t)r.rec;
}

// Per-element constant tables (host-computed).
struct Tables {
  double B[kMaxQ][kMaxM];   // P_j(xi_q)
  double WG[kMaxQ][kMaxM];  // w_q P_j'(xi_q)
  double WB[kMaxQ][kMaxM];  // w_q P_j(xi_q)
  double Dm[kMaxM][kMaxM];  // int P_j' P_k dxi (LDG volume term)
  // the LDG gradient at a point of row r (nodes r < M, then xi = +1, xi = -1) is
  // (GA_r w*_R - GB_r w*_L - sum_k GD_rk w_k)/dx:  GA_r = sum_j (2j+1) P_j(xi_r),
  // GB_r = sum_j (-1)^j (2j+1) P_j(xi_r), GD_rk = sum_j (2j+1) P_j(xi_r) Dm_jk
  double GD[kMaxQ + 2][kMaxM];
  double GA[kMaxQ + 2], GB[kMaxQ + 2];
};

struct OneStep {
  double gamma, q_heat, e_act, k_pre;
};

// Time-integration coefficients of one RK stage.
struct RkStage {
  int two_n;            // 0: Shu-Osher form  out = ca w^n + cb (w^(s) + dt L(w^(s)))  (ca = 0: out = w^(s) + dt L)
                        // 1: 2N form         k = ca k + dt L(u), out = u + cb k
  double ca, cb;
};

// Stages per step of an integrator (0 = SSP-RK3, 1 = RK2, 2 = LSERK4).
__host__ __device__ inline int rk_stages(int rk) { return rk == 0 ? 3 : rk == 1 ? 2 : 5; }

// The coefficients of stage s.  SSP-RK3 in Shu-Osher form; RK2 (Heun) and the
// five-stage fourth-order scheme of Carpenter and Kennedy (NASA TM-109112, 1994)
// in 2N-storage form.
__host__ __device__ inline RkStage rk_stage(int rk, int s) {
  RkStage r{};
  if (rk == 0) {
    r.two_n = 0;
    r.ca = s == 0 ? 0.0 : s == 1 ? 0.75 : 1.0 / 3.0;
    r.cb = s == 0 ? 1.0 : s == 1 ? 0.25 : 2.0 / 3.0;
  } else if (rk == 1) {
    r.two_n = 1;
    r.ca = s == 0 ? 0.0 : -1.0;
    r.cb = s == 0 ? 1.0 : 0.5;
  } else {
    const double A[5] = {0.0, -567301805773.0 / 1357537059087.0, -2404267990393.0 / 2016746695238.0,
                         -3550918686646.0 / 2091501179385.0, -1275806237668.0 / 842570457699.0};
    const double B[5] = {1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
                         1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
                         2277821191437.0 / 14882151754819.0};
    r.two_n = 1;
    r.ca = A[s];
    r.cb = B[s];
  }
  return r;
}

struct EulerArgs {
  const double *w0;     // w^n (may alias wout at the last stage)
  const double *ws;     // stage input w^(s)
  double *wout;         // stage output (unlimited)
  const int *face_if;   // [E+1] interface index of face f, or -1
  // step counters of the two parities: a launch of parity par works on step
  // step[par], and the step's last launch writes step[par ^ 1] = step[par] + 1
  // (plain stores by one workgroup: no launch of the step reads that counter)
  long long *step;
  int par;              // parity of a single-problem launch (batched launches take theirs from the launch)
  int advance;          // this launch ends the time step
  int *err;
  long long target;     // batched launches skip the instance once its step reaches it
  int E;
  int periodic;
  int stage;
  RkStage rk;
  double *kbuf;         // 2N register read by this stage (2N schemes)
  double *kout;         // 2N register written by this stage (kbuf itself without the limiter)
  // batched Shu-Osher stages with the limiter: w^n lives in W[n mod 2] (n = the step
  // counter), stage 1 writes W[1 - n mod 2], stage 2 W[2], stage 3 W[1 - n mod 2], so
  // no stage writes a buffer it reads (the kernel then ignores w0, ws and wout; the
  // single-problem solver passes the same buffers explicitly)
  int alt;
  double *W[3];
  int store_U;          // publish boundary-element outputs for the limiter
  double dt;
  double two_over_dx;
  OneStep ph;
  DelayParams dl;
  RingParams ring;
  Tables tb;
};

// Constants of the troubled-cell indicator and the characteristic WENO limiter
// (Sec. 3.3), which run inside the stage kernel of a limited problem.
struct LimiterArgs {
  int8_t *flags;        // [E] troubled flags of the latest stage
  unsigned long long *flag_count;   // troubled (element, stage) pairs since set_state
  double kx_h;          // dx^((N_p+1)/2)
  int indicator;        // ADG_KXRCF | ADG_MINMOD
  double tvb_mh2;       // M dx^2 of the TVB minmod test
  double gam[3];
  double eps;
  double Bm[kMaxM][kMaxM];    // smoothness-indicator quadratic form
  double Tl[kMaxM][kMaxM];    // re-expansion of the left neighbour in the cell
  double Tr[kMaxM][kMaxM];    // re-expansion of the right neighbour
};

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup b runs on
// XCD b mod 8), each with its own L2.  This maps workgroup b of n to a work item
// so that XCD x gets the contiguous range [x q + min(x, r), ...) of the n items
// (q = n / 8, r = n mod 8): neighbouring items, which share halo data, then meet
// in the same L2.  A bijection of [0, n).
constexpr int kXcds = 8;
__host__ __device__ inline int xcd_item(int b, int n) {
  const int q = n / kXcds, r = n % kXcds;
  const int x = b % kXcds, i = b / kXcds;
  return x * q + (x < r ? x : r) + i;
}

enum ErrBits { kErrState = 1, kErrNewton = 2 };

// Argument blocks of one instance of the one-step model in a batch: one per stage,
// and the limiter constants.
struct EulerSet {
  EulerArgs st[3];
  LimiterArgs lim;
};

// Kernel launchers (defined in the .hip files).
// One stage of the one-step model; `lim` (null = no limiter) adds the limiter to
// the same kernel.
hipError_t launch_euler_stage(int M, int flux, const EulerArgs &a, const LimiterArgs *lim, hipStream_t s);
// Batched one-step stage over a work list of (instance, block) entries, all of
// order M, flux `flux` (Rusanov/HLLC) and limiter choice `lim`, at step counter
// parity `par`.
hipError_t launch_euler_batch(int M, int flux, bool lim, const EulerSet *sets, const int2 *tiles, int ntiles,
                              int stage, int par, hipStream_t s);
// Workgroups of the one-step stage kernel for E elements: a wavefront owns 62
// elements, 60 with the limiter (two halo lanes on each side).
__host__ __device__ inline int euler_blocks(int E, bool lim) {
  const int we = lim ? 60 : 62;
  const int waves = (E + we - 1) / we;
  return (waves + kEulerBlock / 64 - 1) / (kEulerBlock / 64);
}
hipError_t launch_to_planes(const double *src, double *dst, int E, int VM, hipStream_t s);
hipError_t launch_from_planes(const double *src, double *dst, int E, int VM, hipStream_t s);

}  // namespace adg
