// Detailed-chemistry Navier-Stokes stage kernel (LDG): declarations.
#pragma once

#include "adg.h"
#include "adg_internal.hpp"

namespace adg {

// Species capacities of the kernels: a mechanism of Ns species runs in the kernels of the
// smallest capacity that holds it, the species past Ns padded with zero density, no thermo
// and no reactions (they add exact zeros to every species sum and are never stored).
constexpr int kNsMaxSpecies = 9;      // the batched kernels, and single problems with Ns <= 9
constexpr int kNsWideSpecies = 16;    // single problems with 9 < Ns <= 16
constexpr int kNsMaxReactions = 32;
constexpr int kNsBatchReactions = 24;   // reactions of a batched mechanism (rate storage of the batched kernel)
inline int ns_capacity(int n_species) { return n_species <= kNsMaxSpecies ? kNsMaxSpecies : kNsWideSpecies; }

// Mechanism in device memory, read with wave-uniform indices (scalar loads), for kernels of
// species capacity NSC.
template <int NSC>
struct NsMechT {
  static constexpr int kSpecies = NSC;
  int ns, nr;
  double Ru, p_ref, T_guess;
  double mu_ref, ln_T_ref, mu_exp, inv_prandtl;   // mu = mu_ref exp(mu_exp (ln T - ln T_ref))
  double ln_p_over_Ru;              // ln(p_ref / Ru)
  double W[NSC], invW[NSC], Ri[NSC];
  // NASA-7 in Horner-ready form, per species:
  //   cv/R - ... : c0m1 = a0 - 1, a1 .. a4       (cp/R - 1)
  //   (h - R T)/R = T (a0-1 + T (a1/2 + T (a2/3 + T (a3/4 + T a4/5)))) + a5
  //   h/(R T) = a0 + T (a1/2 + ...) + a5 / T
  //   s/R = a0 ln T + T (a1 + T (a2/2 + T (a3/3 + T a4/4))) + a6
  double a[NSC][7];
  double h2[NSC][4];      // a1/2, a2/3, a3/4, a4/5
  double s2[NSC][3];      // a2/2, a3/3, a4/4
  // R_i times the coefficients of the mixture energy quintic (cv/R - 1 form) and R_i:
  // R_i (a0 - 1), R_i a1/2, R_i a2/3, R_i a3/4, R_i a4/5, R_i a5, R_i, 0
  double ek[NSC][8];
  double lnA[kNsMaxReactions], b[kNsMaxReactions], EaR[kNsMaxReactions];
  int dnu[kNsMaxReactions];
  // compact per-reaction form for one lane per (point, reaction): the species
  // multiplied into the forward and reverse rates (-1 = none) and the nonzero
  // net coefficients nu_i = nu''_i - nu'_i with their species, padded to four
  // entries with coefficient 0 (species 0)
  int rf[kNsMaxReactions][2], rr[kNsMaxReactions][2];
  int gidx[kNsMaxReactions][4];
  double gnu[kNsMaxReactions][4];
  // per species, the reactions with a nonzero net coefficient (increasing r) and that
  // coefficient; the entries past the count hold reaction 0 with coefficient 0
  int spn[NSC];
  unsigned char spr[NSC][kNsMaxReactions];
  signed char spnu[NSC][kNsMaxReactions];
  int pad_;
};
using NsMech = NsMechT<kNsMaxSpecies>;
using NsMechWide = NsMechT<kNsWideSpecies>;

struct NsArgs {
  const double *w0;
  const double *ws;
  double *wout;
  double *W[3];         // the three state buffers (batched kernel picks them by stage)
  int M;                // N_p + 1
  int ns;               // species of the problem (the kernel's capacity may be larger)
  int periodic;         // 1: periodic domain; 0: transmissive ends (ghost trace = interior trace)
  const int *face_if;   // [E+1] interface index of face f, or -1
  long long *step;      // step counters of the two parities (as in EulerArgs)
  int par;              // parity of a single-problem launch
  int advance;          // this launch ends the time step
  int *err;
  long long target;     // batched launches skip the instance once its step reaches it
  const void *mech;     // NsMechT<capacity> of the kernel that runs the problem
  // AT combinations carried between launches (single problems; nullptr: gathered in the launch).
  // Record of face f at f * (2 Vg + 1), Vg = 3 + ns: [0, Vg) the AT central traces, [Vg, 2 Vg)
  // the AT fluxes, [2 Vg] the delay (PE-interface faces).  at_in holds this launch's values
  // (written by the previous launch), at_out receives the next launch's (stage + 1 of this
  // step, or stage 0 of the next; nst stages per step).
  const double *at_in;
  double *at_out;
  int nst;
  int E;
  int stage;
  RkStage rk;
  double *kbuf;         // 2N register (2N schemes)
  int viscous;
  double dt;
  double inv_dx;       // 1/dx
  DelayParams dl;
  RingParams ring;
  Tables tb;
};

bool ns_supported(int n_species, int n_reactions);
// Bytes of the device mechanism of a problem with n_species species.
size_t ns_mech_bytes(int n_species);
adg_status ns_setup(NsArgs &a, const adg_physics *ph, const adg_discretization *d, int E, int M, bool periodic,
                    double dx, const DelayParams &dl, const RingParams &rp, const Tables &tb, const int *face_if,
                    long long *step, int *err, void *dev_mech);
// The device form of a mechanism (host side; validates it).
template <int NSC>
adg_status ns_build_mech(const adg_physics *ph, NsMechT<NSC> &hm);
// Work decompositions of the single-problem stage kernel: (tile elements, threads)
// = (8, 512), (8, 256), (4, 256), (4, 512), (8, 1024).
constexpr int kNsConfigs = 5;
// Capacity from a.ns; mixed = FP32 modal operators (for N_p <= 3; N_p = 4 keeps FP64 ones).
hipError_t launch_ns_stage(int M, int cfg, const NsArgs &a, bool mixed, hipStream_t s);
// One stage for every (instance, tile) entry of `tiles` (device), at step counter parity par;
// mixed = FP32 modal operators; max_m = the largest N_p + 1 among the listed instances; tiles
// of tile_elems (4 or 8) elements.
hipError_t launch_ns_batch(const NsArgs *insts, const int2 *tiles, int ntiles, int stage, int par, bool mixed,
                           int max_m, int tile_elems, hipStream_t s);
constexpr int kNsMinTile = 4;

}  // namespace adg
