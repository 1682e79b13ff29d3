// Fused SSP-RK3 stage kernel for the detailed-chemistry Navier-Stokes model
// (Sec. 2 Eq. (1)-(3), Sec. 3.1 LDG form of Eq. (5), Sec. 3.2 AT fluxes).
//
// One workgroup per tile of TE elements (4 or 8), periodic domain.  The tile and a
// halo of two elements on each side are staged in LDS; every later phase reads
// LDS only:
//   1. face traces of w for the tile and halo;
//   2. central traces w* at the faces; at PE interfaces the synchronous w* of
//      this level goes to the history ring and the element-side w* becomes the
//      AT combination of past levels (Eq. (7) applied to w*);
//   3. LDG gradients q (modal) of the tile and one halo element per side;
//   4. a group of lanes per point (quadrature nodes of the tile, both traces of
//      every tile face): temperature Newton, primitives, convective and diffusive
//      fluxes, and at the nodes the Gibbs energies and concentrations (FP64
//      throughout);
//   5. mass-action rates per (node, reaction) and, beside them, the Rusanov total
//      flux per face (at PE interfaces the synchronous flux goes to the ring and
//      the AT combination replaces it); then the species production per (node,
//      species);
//   6. volume and source projection, lift and SSP-RK3 combination; the output
//      is stored once.
#include "adg_device.hpp"
#include "adg_ns.hpp"

#include <cmath>
#include <cstring>
#include <type_traits>

namespace adg {

constexpr int kThreadsBatch = 256;   // batched kernel: more resident workgroups per CU
constexpr int kBatchLanesPerPoint = 4;   // batched kernel: lanes per point of the point phase

// Sum over the LP lanes of a point group (every lane receives the same value:
// the pairwise sums are formed in the same order on every lane).  Groups of up to
// 16 lanes use lane moves inside the SIMD's rows (swap within pairs, then within
// quads; then each lane meets the mirror lane of its half row, then of its row,
// which after the previous steps holds the same partial sum as the lane
// (lane ^ 4), (lane ^ 8) would), wider ones the LDS crossbar.
template <int LP>
__device__ __forceinline__ double group_sum(double x) {
  if constexpr (LP <= 16) {
    if constexpr (LP >= 2) x += dpp_move<kDppXor1>(x);
    if constexpr (LP >= 4) x += dpp_move<kDppXor2>(x);
    if constexpr (LP >= 8) x += dpp_move<kDppHalfMirror>(x);
    if constexpr (LP >= 16) x += dpp_move<kDppMirror>(x);
  } else {
#pragma unroll
    for (int m = 1; m < LP; m <<= 1) x += __shfl_xor(x, m, LP);
  }
  return x;
}

// Temperature from the internal energy e* by Newton's method from the fixed
// start T_guess, at most 50 iterations.  The mixture energy sum_i Y_i e_i(T) is
// linear in the species, so it is one quintic
// e(T) = T (c0 + T (c1 + T (c2 + T (c3 + T c4)))) + c5; returns cv(T) too.
// Newton converges quadratically here (cv > 0 varies slowly with T): once a
// correction is below 1e-8 T the iterate it produces is within about 1e-16 T of
// the root, so the loop stops there, one iteration before a correction below
// 1e-12 T would show it.
__device__ __forceinline__ bool newton_T(const double (&c)[6], double T0, double estar, double &T, double &cv) {
  const double d1 = 2.0 * c[1], d2 = 3.0 * c[2], d3 = 4.0 * c[3], d4 = 5.0 * c[4];
  T = T0;
  bool conv = false;
  for (int it = 0; it < 50; ++it) {
    const double e = T * (c[0] + T * (c[1] + T * (c[2] + T * (c[3] + T * c[4])))) + c[5];
    const double cvi = c[0] + T * (d1 + T * (d2 + T * (d3 + T * d4)));
    const double dT = (e - estar) * __builtin_amdgcn_rcp(cvi);   // the correction needs no IEEE quotient
    T -= dT;
    if (!(T > 0.0) || !isfinite(T)) break;
    if (fabs(dT) <= 1e-8 * T) { conv = true; break; }
  }
  cv = c[0] + T * (d1 + T * (d2 + T * (d3 + T * d4)));
  return conv;
}

// LDS arena of one tile.
template <int M, int NS, int TE, int NRC = kNsMaxReactions>
struct NsLds {
  static constexpr int V = 3 + NS, Q = M;
  static constexpr int NH = TE + 4;   // tile + 2 halo elements per side; local l <-> element e0 - 2 + l
  static constexpr int NF = TE + 3;   // faces e0-1 .. e0+TE+1; local fl <-> face e0 - 1 + fl
  static constexpr int NN = TE * Q;   // quadrature nodes of the tile; node p <-> element p / Q, node p % Q
  static constexpr int NP = NN + 2 * (TE + 1);   // points: the nodes, then the face traces
  static constexpr int NR = NRC;   // reaction capacity of the rate storage
  // rows padded to an odd number of doubles: the lanes of a point group read or write one
  // row each (their species) at the same column, and rows an even number of doubles apart
  // would put several of them on the same LDS banks
  static constexpr int NHP = NH | 1, NNP = NN | 1, NPP = NP | 1;
  double sW[V * M][NHP];
  double sTm[V][NHP], sTp[V][NHP];
  double sG[V][NNP];
  // the central traces are last read by the point phase (synchronous gradient traces); the
  // species production takes their place
  union {
    struct {
      double sWc[V][NF], sWa[V][NF];
    } c;
    double sS[NS][NNP];
  } u0;
  // the species sums of the mixture energy polynomial are read by the mixture chain before the
  // concentrations and Gibbs energies are formed
  union {
    double sMix[8][NPP];   // sums over species of Y_i/rho-weighted coefficients; row 7: e*
    struct {
      double sConc[NS][NNP], sGRT[NS][NNP];
    } g;
  } u1;
  // values and gradients at the points and the per-point results of the mixture chain are dead
  // once the point phase has ended: the reaction rates of the chemistry phase take their place
  union {
    struct {
      double sX[V][NNP];    // values at the nodes (those at the face traces are sTm / sTp)
      double sDx[V][NPP];   // gradients at the points
      double sRinv[NPP], sU[NPP], sRhoD[NPP], sKc[NPP];   // 1/rho, u, rho D, kappa / c_v
    } p;
    double sRate[NR][NN];
  } u;
  double sGf[2][V][TE + 1], sGs[2][V][TE + 1];
  double sLam[2][TE + 1];
  double sTT[NPP], sLnT[NPP], sInvT[NPP];
  double sF[V][TE + 1], sFat[V][TE + 1];
  // operator tables, indexed at run time (copied whole): nodal values, volume and source
  // projections, gradients at the points (rows: the nodes, then xi = +1 and xi = -1)
  Tables sTb;
  int sI[NF], sK[NF];
};

// AT combination (Eq. (7)) of the central trace and the flux of variable v at interface i from
// the levels n-k .. n-k-q+1 of stage st: levels 0..3 given (w, f; a level past q holds level
// n-k and has weight 0), later ones (q > 4) read here one at a time.  The carried and the
// in-launch combinations both come from here, so they round alike.
__device__ __forceinline__ void at_combine(const NsArgs &a, int q, int k, int nmod, int st, int i, int v,
                                           const double (&w)[4], const double (&f)[4], double &acw, double &acf) {
  acw = 0.0;
  acf = 0.0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const double c = j < q ? at_weight(q, k, j) : 0.0;
    acw += c * w[j];
    acf += c * f[j];
  }
  for (int j = 4; j < q; ++j) {
    const double c = at_weight(q, k, j);
    const double *rec = ring_at(a.ring, ring_slot(nmod, k + j, a.ring.D), st, a.dl.nif, i);
    acw += c * rec[a.ring.off_Wc + v];
    acf += c * rec[a.ring.off_F + v];
  }
}

// One tile of one stage (all phases).  OpT is the arithmetic type of the modal
// operators (interpolation to nodes and traces, LDG gradient, volume integral):
// double for the plain path, float for the mixed-precision path.  Point physics
// (temperature Newton, fluxes, transport, chemistry), face averages, the source
// projection and the RK update are FP64 in both.
//
// The mixed path contracts in FP32 only what is small against the element's
// own level: P_0 = 1, so nodal values and traces are mode 0 (FP64) plus the
// FP32 sum of the higher modes; the volume integral uses
// sum_q w_q P_j'(xi_q) = P_j(1) - P_j(-1) to integrate the deviation of the
// flux from its value at the first node in FP32 and the rest in FP64; the LDG
// gradient likewise takes the element mean out of its face and volume terms.
// The FP32 rounding then scales with the variation inside an element, not with
// the magnitude of the state (pressure-sized fluxes would otherwise lose about
// 4 digits of their element-to-element differences).  Gradients at nodes and
// traces are likewise mode 0 plus the FP32 sum of the higher modes.
// LPP: lanes per point of the point phase (0: the workgroup's lanes spread over
// 32 or 64 point slots).
template <int M, int NS, typename OpT, int NTH, int TE, int LPP = 0, int NRC = kNsMaxReactions>
__device__ __forceinline__ void ns_tile(const NsArgs &a, const double *__restrict__ ws, const double *w0,
                                        double *wout, int stage, int advance, const RkStage rk, double *kbuf,
                                        int e0, int par,
                                        NsLds<M, NS, TE, NRC> &Ls, NsMechT<NS> &smech) {
  constexpr int V = 3 + NS, Q = M;
  using Lds = NsLds<M, NS, TE, NRC>;
  constexpr int NH = Lds::NH, NF = Lds::NF, NN = Lds::NN;
  auto &sW = Ls.sW;
  auto &sTm = Ls.sTm;
  auto &sTp = Ls.sTp;
  auto &sWc = Ls.u0.c.sWc;
  auto &sWa = Ls.u0.c.sWa;
  auto &sS = Ls.u0.sS;
  auto &sX = Ls.u.p.sX;
  auto &sDx = Ls.u.p.sDx;
  auto &sRinv = Ls.u.p.sRinv;
  auto &sU = Ls.u.p.sU;
  auto &sRhoD = Ls.u.p.sRhoD;
  auto &sKc = Ls.u.p.sKc;
  auto &sTT = Ls.sTT;
  auto &sG = Ls.sG;
  auto &sMix = Ls.u1.sMix;
  auto &sConc = Ls.u1.g.sConc;
  auto &sGRT = Ls.u1.g.sGRT;
  auto &sRate = Ls.u.sRate;
  auto &sGf = Ls.sGf;
  auto &sGs = Ls.sGs;
  auto &sLam = Ls.sLam;
  auto &sLnT = Ls.sLnT;
  auto &sInvT = Ls.sInvT;
  auto &sF = Ls.sF;
  auto &sFat = Ls.sFat;
  auto &sWG = Ls.sTb.WG;
  auto &sWB = Ls.sTb.WB;
  auto &sGD = Ls.sTb.GD;
  auto &sGA = Ls.sTb.GA;
  auto &sGB = Ls.sTb.GB;
  auto &sI = Ls.sI;
  auto &sK = Ls.sK;
  constexpr int NP = Lds::NP;
  constexpr bool kMixed = !std::is_same<OpT, double>::value;

  const int t = threadIdx.x;
  const int E = a.E;
  const int nloc = min(TE, E - e0);
  const NsMechT<NS> *__restrict__ mk = &smech;
  // variables stored per element in HBM and in the ring (the capacity NS may pad species)
  const int Vg = 3 + a.ns, VMg = Vg * M;
  const bool periodic = a.periodic != 0;
  const int q_at = a.dl.q;
  bool ok = true;

  // 0. mechanism, operator tables, state of the tile and its halo, PE-interface data of the
  //    faces, then the traces, the nodal values, the central traces and the AT combinations of
  //    past levels (Eq. (7)) formed from the loaded registers.  Every global load is issued
  //    first, and nothing before them depends on a loaded value (the step counter included),
  //    so the phase costs about one memory latency plus the arithmetic of its lanes.
  constexpr int kOut = (V * M * TE + NTH - 1) / NTH;
  // the second operand of the RK combination (w^n, or the 2N register) of the outputs
  // this thread writes in the last phase
  const bool use_prev = rk.two_n ? rk.ca != 0.0 : rk.ca != 0.0 || rk.cb != 1.0;
  const double *prev = rk.two_n ? kbuf : w0;
  double w0pre[kOut];
  long long n;
  // element items: lane jw of wavefront w < kEW holds variable w * VPW + jw / NH at local
  // element el = jw % NH (element e0 - 2 + el), so the NH elements of a variable sit in
  // consecutive lanes of one wavefront.  It loads the element's modes, forms its traces and,
  // inside the tile, its nodal values, and owns the face right of it (face fl = el, between
  // local elements el and el + 1, for el < NF): the next lane's left trace completes the
  // central trace, and the item gathers the face's past levels.
  constexpr int VPW = 64 / NH;   // variables per wavefront
  constexpr int kEW = (V + VPW - 1) / VPW;
  static_assert(kEW * 64 <= NTH, "one element item per lane");
  {
    constexpr int nwords = (int)(sizeof(NsMechT<NS>) / 8);
    constexpr int kMw = (nwords + NTH - 1) / NTH;
    constexpr int twords = (int)(sizeof(Tables) / 8);
    constexpr int kTw = (twords + NTH - 1) / NTH;
    const unsigned long long *src = reinterpret_cast<const unsigned long long *>(a.mech);
    unsigned long long *dst = reinterpret_cast<unsigned long long *>(&smech);
    const unsigned long long *tsrc = reinterpret_cast<const unsigned long long *>(&a.tb);
    unsigned long long *tdst = reinterpret_cast<unsigned long long *>(&Ls.sTb);
    unsigned long long mw[kMw], tw[kTw];
    const int jw = t & 63;
    const int ev = (t >> 6) * VPW + jw / NH, el = jw % NH;
    const bool eitem = t < kEW * 64 && jw < VPW * NH && ev < V;
    const bool real = eitem && ev < Vg;   // a stored variable (padded species stay zero)
    const bool hasface = eitem && el < NF;
    // the interface of the item's face: loaded first, so the history loads that depend on it
    // need not wait for the state
    int gfi = -1, gk = 0;
    double gkc = 0.0;
    double g_w[4], g_f[4];
    if (hasface && real) {
      int f = e0 - 1 + el;
      if (periodic) {
        while (f < 0) f += E;
        while (f >= E) f -= E;
      }
      if (f >= 0 && f <= E) {
        gfi = a.face_if[f];
        if (a.at_in) {
          // carried from the previous launch: no dependence on the interface index
          const double *rec = a.at_in + (size_t)f * (2 * Vg + 1);
          g_w[0] = rec[ev];
          g_f[0] = rec[Vg + ev];
          gkc = rec[2 * Vg];
        }
      }
    }
#pragma unroll
    for (int m = 0; m < kMw; ++m) {
      const int idx = t + m * NTH;
      mw[m] = idx < nwords ? src[idx] : 0ull;
    }
#pragma unroll
    for (int m = 0; m < kTw; ++m) {
      const int idx = t + m * NTH;
      tw[m] = idx < twords ? tsrc[idx] : 0ull;
    }
    // at a transmissive end the ghost element beyond a boundary face carries the interior trace
    // at that face on both of its sides (ghost trace = interior trace), so its lane loads the
    // interior element; elements further out are never read
    int ghost = 0, esrc = e0 - 2 + el;
    if (!periodic) {
      if (esrc < 0) { ghost = esrc == -1 ? 1 : 3; esrc += 1; }
      else if (esrc >= E) { ghost = esrc == E ? 2 : 3; esrc -= 1; }
    } else {
      // within a few periods of [0, E)
      while (esrc < 0) esrc += E;
      while (esrc >= E) esrc -= E;
    }
    double wl[M];
#pragma unroll
    for (int j = 0; j < M; ++j) {
      wl[j] = 0.0;
      if (real && ghost != 3) wl[j] = ws[sidx(esrc, ev * M + j, VMg)];
    }
    int fi = -1;
    double kc = 0.0;   // the carried delay of the face
    if (t < NF) {
      int f = e0 - 1 + t;
      if (periodic) {
        while (f < 0) f += E;
        while (f >= E) f -= E;
      }
      fi = f >= 0 && f <= E ? a.face_if[f] : -1;
      if (a.at_in && f >= 0 && f <= E) kc = a.at_in[(size_t)f * (2 * Vg + 1) + 2 * Vg];
    }
#pragma unroll
    for (int m = 0; m < kOut; ++m) {
      const int idx = t + m * NTH;
      const int c = idx / TE, el2 = idx % TE;
      w0pre[m] = 0.0;
      if (use_prev && idx < V * M * TE && el2 < nloc && c < VMg) w0pre[m] = prev[sidx(e0 + el2, c, VMg)];
    }
    n = a.step[par];
    const int nm = step_mod(n, a.ring.D);   // the current level's ring slot
    // the carried delays are first used here, after every load has been issued (left to itself
    // the compiler converts them to int right after their loads, which waits for those loads
    // before the rest are issued)
    asm volatile("" : "+v"(gkc), "+v"(kc));
    // levels 0..3 of the item's face (a level past q reads level n-k with weight 0); they land
    // while the items form their traces and nodal values.  Carried: the previous launch drew
    // the delay (a step before q, which has no predecessor after a reset, has only zero delays).
    if (gfi >= 0) {
      if (a.at_in) {
        gk = n >= q_at ? (int)gkc : 0;
      } else {
        gk = eff_delay<true>(a.dl, n, gfi);
        if (gk > 0) {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const double *rec = ring_at(a.ring, ring_slot(nm, gk + (j < q_at ? j : 0), a.ring.D), stage, a.dl.nif, gfi);
            g_w[j] = rec[a.ring.off_Wc + ev];
            g_f[j] = rec[a.ring.off_F + ev];
          }
        }
      }
    }
#pragma unroll
    for (int m = 0; m < kMw; ++m) {
      const int idx = t + m * NTH;
      if (idx < nwords) dst[idx] = mw[m];
    }
#pragma unroll
    for (int m = 0; m < kTw; ++m) {
      const int idx = t + m * NTH;
      if (idx < twords) tdst[idx] = tw[m];
    }
    if (t < NF) {
      sI[t] = fi;
      sK[t] = fi < 0 ? 0 : a.at_in ? (n >= q_at ? (int)kc : 0) : eff_delay<true>(a.dl, n, fi);
    }
    // traces, nodal values and central traces of the element items: every lane of their
    // wavefronts takes part in the lane move (lanes without an item hold zeros)
    if (t < kEW * 64) {
      OpT sm = 0, sp = 0;
#pragma unroll
      for (int j = kMixed ? 1 : 0; j < M; ++j) {
        const OpT c = (OpT)wl[j];
        sp += c;
        sm += (j & 1) ? -c : c;
      }
      double tm, tp;
      if constexpr (kMixed) {
        tm = wl[0] + (double)sm;
        tp = wl[0] + (double)sp;
      } else {
        tm = (double)sm;
        tp = (double)sp;
      }
      if (ghost == 1) tp = tm;
      else if (ghost == 2) tm = tp;
      else if (ghost == 3) tm = tp = 0.0;
      const double tm_right = dpp_move<kDppFromNext>(tm);   // left trace of element el + 1
      if (eitem) {
#pragma unroll
        for (int j = 0; j < M; ++j) sW[ev * M + j][el] = ghost ? 0.0 : wl[j];
        sTm[ev][el] = tm;
        sTp[ev][el] = tp;
        if (el >= 2 && el < TE + 2) {
#pragma unroll
          for (int qn = 0; qn < Q; ++qn) {
            OpT xo = 0;
#pragma unroll
            for (int j = kMixed ? 1 : 0; j < M; ++j) xo += (OpT)a.tb.B[qn][j] * (OpT)wl[j];
            sX[ev][(el - 2) * Q + qn] = kMixed ? wl[0] + (double)xo : (double)xo;
          }
        }
      }
      if (hasface) {
        // central trace; the synchronous one of a PE interface is published for this level
        // (faces e0 .. e0+nloc-1 are owned by this tile).  The AT combination of the face's
        // gathered levels takes its place at a delayed PE interface.
        const double wc = kMixed ? 0.5 * (tp + tm_right) : (double)((OpT)0.5 * ((OpT)tp + (OpT)tm_right));
        sWc[ev][el] = wc;
        double wa = wc;
        if (!real) {   // padded species: nothing in the ring
          wa = 0.0;
          if (el >= 1 && el <= TE + 1) sFat[ev][el - 1] = 0.0;
        } else if (gfi >= 0) {
          if (el >= 1 && el <= nloc) ring_at(a.ring, nm, stage, a.dl.nif, gfi)[a.ring.off_Wc + ev] = wc;
          if (gk > 0) {
            double acw, acf;
            if (a.at_in) {
              acw = g_w[0];
              acf = g_f[0];
            } else {
              at_combine(a, q_at, gk, nm, stage, gfi, ev, g_w, g_f, acw, acf);
            }
            wa = acw;
            if (el >= 1 && el <= TE + 1) sFat[ev][el - 1] = acf;
          }
        }
        sWa[ev][el] = wa;
      }
    }
  }
  const int nmod = step_mod(n, a.ring.D);   // the current level's ring slot
  __syncthreads();
  const int nr = mk->nr;

  // face trace point p >= NN: face e0 + ff, side (0: the element left of the face, at its
  // xi = +1) and the side es whose element is evaluated (at a transmissive end the ghost side
  // takes the interior's trace and gradient trace)
  auto trace_side = [&](int p, int &ff, int &side, int &es) {
    const int pp = p - NN;
    ff = pp >> 1;
    side = pp & 1;
    es = side;
    if (!periodic) {
      if (e0 + ff == 0 && side == 0) es = 1;
      else if (e0 + ff == E && side == 1) es = 0;
    }
  };
  // gradient slot lq (elements e0 - 1 + lq; faces lq and lq + 1) of the element evaluated at
  // point p, and the row r of p in the point tables
  auto point_slot = [&](int p, int &lq, int &r) {
    if (p < NN) {
      lq = p / Q + 1;
      r = p % Q;
    } else {
      int ff, side, es;
      trace_side(p, ff, side, es);
      lq = ff + es;
      r = Q + es;
    }
  };

  // the values of the variables at point p: the nodal values, or the traces of the side
  // evaluated; variable v is at [v * stride] of the returned row
  auto values = [&](int p, int &stride) -> const double * {
    if (p < NN) {
      stride = Lds::NNP;
      return &sX[0][p];
    }
    int ff, side, es;
    trace_side(p, ff, side, es);
    stride = Lds::NHP;
    return es ? &sTm[0][ff + 1 + es] : &sTp[0][ff + 1 + es];
  };
  // 2. the species sums of the mixture chain: the internal energy
  //    e(T) = sum_i Y_i R_i [T (a_i0 - 1 + T (a_i1/2 + ...)) + a_i5] is one quintic in T whose
  //    coefficients are rho^-1 sum_i rho_i R_i (a_i0 - 1), ..., and R = rho^-1 sum_i rho_i R_i
  //    (rows 0..6); row 7 holds e* = E/rho - u^2/2 (with 1/rho and u beside it).  The sums take
  //    the first lanes and the gradients of the next step the last ones, laid out so that where
  //    the workgroup has the lanes no lane forms both: one lane per (point, row) (layout 0);
  //    one per (point, rows g and g + 4) for g < 3, one per (point, row 3) and one per
  //    (point, row 7) (layout 1); else one per (point, rows g and g + 4), the g = 3 lane also
  //    forming row 7 (layout 2).  A lane reads the point's species once for its rows.
  constexpr int VH1 = V, VH2 = (V + 1) / 2, VH3 = (V + 2) / 3;
  constexpr bool kFit0 = 8 * NP + VH1 * NP <= NTH;
  constexpr int kFit1 = 5 * NP + VH1 * NP <= NTH ? 1 : 5 * NP + VH2 * NP <= NTH ? 2 : 5 * NP + VH3 * NP <= NTH ? 3 : 0;
  constexpr int kMixLayout = kFit0 ? 0 : kFit1 ? 1 : 8 * NP <= NTH ? 0 : 2;
  // variables per lane of the gradients
  constexpr int VPL = kFit0 ? 1 : kFit1 ? kFit1 : V * NP > NTH ? 2 : 1;
  auto mixture_row7 = [&](int p, const double *vrow, int vs) {
    const double rho_inv = 1.0 / vrow[0];
    const double u = vrow[vs] * rho_inv;
    sRinv[p] = rho_inv;
    sU[p] = u;
    sMix[7][p] = vrow[2 * vs] * rho_inv - 0.5 * u * u;
  };
  if constexpr (kMixLayout == 0) {
    if (t < 8 * NP) {
      const int q = t / NP, p = t % NP;
      int vs;
      const double *vrow = values(p, vs);
      if (q == 7) {
        mixture_row7(p, vrow, vs);
      } else {
        double sum = 0.0;
#pragma unroll
        for (int i = 0; i < NS; ++i) sum += vrow[(3 + i) * vs] * mk->ek[i][q];
        sMix[q][p] = sum;
      }
    }
  } else if constexpr (kMixLayout == 1) {
    if (t < 5 * NP) {
      const int g = t / NP, p = t % NP;
      int vs;
      const double *vrow = values(p, vs);
      if (g == 4) {
        mixture_row7(p, vrow, vs);
      } else {
        double lo = 0.0, hi = 0.0;
#pragma unroll
        for (int i = 0; i < NS; ++i) {
          const double x = vrow[(3 + i) * vs];
          lo += x * mk->ek[i][g];
          if (g < 3) hi += x * mk->ek[i][g + 4];
        }
        sMix[g][p] = lo;
        if (g < 3) sMix[g + 4][p] = hi;
      }
    }
  } else {
    for (int idx = t; idx < 4 * NP; idx += NTH) {
      const int g = idx / NP, p = idx % NP;
      int vs;
      const double *vrow = values(p, vs);
      double lo = 0.0, hi = 0.0;
#pragma unroll
      for (int i = 0; i < NS; ++i) {
        const double x = vrow[(3 + i) * vs];
        lo += x * mk->ek[i][g];
        if (g < 3) hi += x * mk->ek[i][g + 4];
      }
      sMix[g][p] = lo;
      if (g < 3) sMix[g + 4][p] = hi;
      else mixture_row7(p, vrow, vs);
    }
  }

  // 3. gradients at the points, in the same phase as the species sums: both read only what the
  //    load phase wrote, and neither reads what the other writes.  The LDG gradient of the
  //    element with gradient slot lq (left face lq, right face lq + 1) has modes
  //    q_j = (2j+1)/dx [w*_R - (-1)^j w*_L - sum_k D_jk w_k];
  //    its value at a point of row r (node r < Q, the right end xi = +1 for r = Q, the left end
  //    for r = Q + 1) is sum_j P_j(xi_r) q_j = (A_r w*_R - B_r w*_L - sum_k G_rk w_k)/dx, with the
  //    tabulated A_r = sum_j (2j+1) P_j(xi_r), B_r = sum_j (-1)^j (2j+1) P_j(xi_r) and
  //    G_rk = sum_j (2j+1) P_j(xi_r) D_jk.  Since D_j0 = 1 - (-1)^j, A_r - B_r = G_r0 and the mean
  //    cancels: the mixed path forms the face terms against it in FP64 and the rest in FP32.
  //    A lane forms the gradients of VPL variables (v, v + VH, ...) at its point, reading the
  //    point's table row once; where the lanes suffice for both the items are taken from the
  //    last lane down, clear of the sums.
  {
    constexpr int VH = (V + VPL - 1) / VPL;
    constexpr bool kFromTop = kFit0 || kFit1 != 0;
    for (int idx = kFromTop ? NTH - 1 - t : t; idx < VH * NP; idx += NTH) {
      const int h = idx / NP, p = idx % NP;
      int lq, r;
      point_slot(p, lq, r);
      double gd[M];
#pragma unroll
      for (int k = 0; k < M; ++k) gd[k] = sGD[r][k];
      const double ga = sGA[r], gb = sGB[r];
#pragma unroll
      for (int u = 0; u < VPL; ++u) {
        const int v = h + u * VH;
        if (v >= V) break;
        double d;
        if constexpr (kMixed) {
          const double m0 = sW[v * M][lq + 1];
          OpT vol = 0;
#pragma unroll
          for (int k = 1; k < M; ++k) vol += (OpT)gd[k] * (OpT)sW[v * M + k][lq + 1];
          d = a.inv_dx * (ga * (sWa[v][lq + 1] - m0) - gb * (sWa[v][lq] - m0) - (double)vol);
        } else {
          double vol = 0.0;
#pragma unroll
          for (int k = 0; k < M; ++k) vol += gd[k] * sW[v * M + k][lq + 1];
          d = a.inv_dx * (ga * sWa[v][lq + 1] - gb * sWa[v][lq] - vol);
        }
        sDx[v][p] = d;
      }
    }
  }
  __syncthreads();

  // 4. point physics (FP64).  Points: the quadrature nodes of the tile, then both traces of the
  //    faces e0 .. e0+TE.  First one lane per point forms the mixture chain (species sums of
  //    the energy polynomial, temperature Newton, pressure, sound speed, transport
  //    coefficients, the convective and non-species diffusive fluxes); then a group of LP lanes
  //    per point shares the species (diffusive species and enthalpy fluxes, Gibbs energies and
  //    concentrations at the nodes), reducing the two species sums of the heat flux over the
  //    group.
  //    At a PE interface the synchronous gradient trace adds to the point's gradient the
  //    difference that the synchronous central traces (instead of the AT ones) make to it.
  auto pe_corr = [&](int v, int lq, int r) -> double {
    const double dl = sWc[v][lq] - sWa[v][lq], dr = sWc[v][lq + 1] - sWa[v][lq + 1];
    return a.inv_dx * (sGA[r] * dr - sGB[r] * dl);
  };
  static_assert(NTH - 64 >= V * TE, "a lane of the later wavefronts per (variable, owned face)");
  if (t >= 64 && a.at_out) {
    // the wavefronts the mixture chain leaves idle form the next launch's AT combinations at the
    // PE interfaces this tile owns (faces e0 .. e0+nloc-1): stage + 1 of this step, or stage 0
    // of the next; their levels all precede what this launch writes
    const int idx = t - 64;
    const int v = idx / TE, fo = idx % TE;
    const int i = sI[fo + 1];
    if (v < Vg && fo < nloc && i >= 0) {
      const bool last = stage == a.nst - 1;
      const long long n2 = n + (last ? 1 : 0);
      const int s2 = last ? 0 : stage + 1;
      const int k2 = eff_delay<true>(a.dl, n2, i);
      const size_t base = (size_t)(e0 + fo) * (2 * Vg + 1);
      if (v == 0) a.at_out[base + 2 * Vg] = (double)k2;
      if (k2 > 0) {
        const int nm2 = step_mod(n2, a.ring.D);
        double w[4], f[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const double *rec = ring_at(a.ring, ring_slot(nm2, k2 + (j < q_at ? j : 0), a.ring.D), s2, a.dl.nif, i);
          w[j] = rec[a.ring.off_Wc + v];
          f[j] = rec[a.ring.off_F + v];
        }
        double acw, acf;
        at_combine(a, q_at, k2, nm2, s2, i, v, w, f, acw, acf);
        a.at_out[base + v] = acw;
        a.at_out[base + Vg + v] = acf;
      }
    }
  }
  if (t < NP) {
    const int p = t;
    const bool node = p < NN;
    int lq, r;
    point_slot(p, lq, r);
    int ff = 0, side = 0, es = 0;
    if (!node) trace_side(p, ff, side, es);
    const bool valid = periodic || (node ? p / Q < nloc : e0 + ff <= E);
    const bool pe = !node && sI[ff + 1] >= 0;
    int vs;
    const double *vrow = values(p, vs);
    const double wr = vrow[0], wm = vrow[vs], we = vrow[2 * vs];
    const double rho_inv = sRinv[p], u = sU[p], estar = sMix[7][p];
    double c[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) c[q] = sMix[q][p] * rho_inv;
    const double Rmix = sMix[6][p] * rho_inv;
    double T, cv;
    const bool conv = newton_T(c, mk->T_guess, estar, T, cv);
    const double lnT = log(T);   // shared by the viscosity law and the Gibbs energies
    const double cp = cv + Rmix;
    const double pr = wr * Rmix * T;
    const double rcv = 1.0 / cv;
    const double snd = sqrt(cp * rcv * pr * rho_inv);
    if (valid) ok = conv && pr > 0.0 && isfinite(pr) && wr > 0.0 && ok;
    double g1 = wm * u + pr, g2 = u * (we + pr);
    double gs1 = g1, gs2 = g2;
    double rhoD = 0.0, kc = 0.0;
    if (a.viscous) {
      // f^d of Eq. (2)-(3) without its species sums: tau = 4/3 mu u_x and the heat flux
      // -kappa T_x with T_x = (e_x - sum_i e_i dY_i/dx)/c_v; the species terms (unit Lewis
      // number, J_i = -rho D dY_i/dx, rho D = mu/Pr) are added by the species lanes
      const double mu = mk->mu_ref * exp(mk->mu_exp * (lnT - mk->ln_T_ref));
      const double kappa = mu * cp * mk->inv_prandtl;
      rhoD = mu * mk->inv_prandtl;
      kc = kappa * rcv;
      const double En = we * rho_inv;
      auto partial = [&](double d0, double d1, double d2, double &h1, double &h2) {
        const double u_x = (d1 - u * d0) * rho_inv;
        const double e_x = (d2 - En * d0) * rho_inv - u * u_x;
        const double tau = (4.0 / 3.0) * mu * u_x;
        h1 -= tau;
        h2 -= tau * u + kc * e_x;
      };
      partial(sDx[0][p], sDx[1][p], sDx[2][p], g1, g2);
      if (pe)
        partial(sDx[0][p] + pe_corr(0, lq, r), sDx[1][p] + pe_corr(1, lq, r), sDx[2][p] + pe_corr(2, lq, r), gs1,
                gs2);
    }
    if (valid) {
      if (node) {
        sG[0][p] = wm;
        sG[1][p] = g1;
        sG[2][p] = g2;
      } else {
        sGf[side][0][ff] = wm;
        sGf[side][1][ff] = g1;
        sGf[side][2][ff] = g2;
        sLam[side][ff] = fabs(u) + snd;
        if (pe) {
          sGs[side][0][ff] = wm;
          sGs[side][1][ff] = gs1;
          sGs[side][2][ff] = gs2;
        }
      }
      sRhoD[p] = rhoD;
      sKc[p] = kc;
      sTT[p] = T;
      sLnT[p] = lnT;
      sInvT[p] = 1.0 / T;
    }
  }
  __syncthreads();
  {
    constexpr int kSlots = NP <= 32 ? 32 : 64;   // point slots per workgroup
    constexpr int LP = LPP > 0 ? LPP : NTH / kSlots;   // lanes per point
    static_assert(LP >= 1 && LP <= 64 && (LP & (LP - 1)) == 0 && NP <= NTH / LP, "every point has a lane group");
    constexpr int NO = (NS + LP - 1) / LP;
    // a wavefront whose lanes all lie past the last point's group has no point to form
    if ((t & ~63) / LP < NP) {
      const int k = t % LP;
      const int p = min(t / LP, NP - 1);          // spare groups redo the last point and write nothing
      const bool node = p < NN;
      int lq, r;
      point_slot(p, lq, r);
      int ff = 0, side = 0, es = 0;
      if (!node) trace_side(p, ff, side, es);
      const bool writer = t / LP < NP && (periodic || (node ? p / Q < nloc : e0 + ff <= E));
      const bool pe = !node && sI[ff + 1] >= 0;
      const double rho_inv = sRinv[p], u = sU[p], T = sTT[p];
      int vs;
      const double *vrow = values(p, vs);
      double gy[NO], gsy[NO], hT[NO], wy[NO];
#pragma unroll
      for (int m = 0; m < NO; ++m) {
        const int i = k + LP * m;
        wy[m] = i < NS ? vrow[(3 + i) * vs] : 0.0;
        gy[m] = gsy[m] = wy[m] * u;
        hT[m] = 0.0;
        if (i < NS) {
          const double *ai = mk->a[i];
          const double *h2i = mk->h2[i];
          hT[m] = T * (ai[0] + T * (h2i[0] + T * (h2i[1] + T * (h2i[2] + T * h2i[3])))) + ai[5];  // h_i/R_i
        }
      }
      if (a.viscous) {
        const double rhoD = sRhoD[p], kc = sKc[p];
        auto species = [&](double d0, bool sync, double (&gyy)[NO]) -> double {
          double sum_eY = 0.0, sum_hJ = 0.0;
#pragma unroll
          for (int m = 0; m < NO; ++m) {
            const int i = k + LP * m;
            if (i >= NS) continue;
            const double dy = sDx[3 + i][p] + (sync ? pe_corr(3 + i, lq, r) : 0.0);
            const double Yx = (dy - (wy[m] * rho_inv) * d0) * rho_inv;
            sum_eY += mk->Ri[i] * (hT[m] - T) * Yx;
            const double J = -rhoD * Yx;
            sum_hJ += mk->Ri[i] * hT[m] * J;
            gyy[m] += J;                  // f^d_i = -J_i
          }
          // heat flux -kappa T_x + sum_i h_i J_i: the part left out of the mixture chain
          return kc * group_sum<LP>(sum_eY) + group_sum<LP>(sum_hJ);
        };
        const double q = species(sDx[0][p], false, gy);
        const double qs = pe ? species(sDx[0][p] + pe_corr(0, lq, r), true, gsy) : 0.0;
        if (writer && k == 0) {
          if (node) {
            sG[2][p] += q;
          } else {
            sGf[side][2][ff] += q;
            if (pe) sGs[side][2][ff] += qs;
          }
        }
      }
      if (writer) {
        if (node) {
          const double invT = sInvT[p], lnT = sLnT[p];
#pragma unroll
          for (int m = 0; m < NO; ++m) {
            const int i = k + LP * m;
            if (i >= NS) continue;
            sG[3 + i][p] = gy[m];
            const double *ci = mk->a[i];
            const double *s2i = mk->s2[i];
            const double sR = ci[0] * lnT + T * (ci[1] + T * (s2i[0] + T * (s2i[1] + T * s2i[2]))) + ci[6];
            sGRT[i][p] = hT[m] * invT - sR;
            sConc[i][p] = wy[m] * mk->invW[i];
          }
        } else {
#pragma unroll
          for (int m = 0; m < NO; ++m) {
            const int i = k + LP * m;
            if (i >= NS) continue;
            sGf[side][3 + i][ff] = gy[m];
            if (pe) sGs[side][3 + i][ff] = gsy[m];
          }
        }
      }
    }
  }
  __syncthreads();

  // chemistry (Sec. 2: W_i omega_i): one lane per (node, reaction), then one lane per (node, species).
  // The rate of one (node, reaction) is branch-free (the unused entries of a reaction's Gibbs
  // list hold coefficient 0, a missing reactant or product multiplies by 1), so a lane forms
  // two of them side by side and their dependent chains overlap.
  {
    auto rate = [&](int idx) -> double {
      const int r = idx / NN, p = idx % NN;
      const double lnT = sLnT[p];
      const double lnkf = mk->lnA[r] + mk->b[r] * lnT - mk->EaR[r] * sInvT[p];
      double dG = 0.0;
#pragma unroll
      for (int g = 0; g < 4; ++g) dG += mk->gnu[r][g] * sGRT[mk->gidx[r][g]][p];
      const double lnKc = -dG + (double)mk->dnu[r] * (mk->ln_p_over_Ru - lnT);
      double fwd = exp(lnkf), rev = exp(lnkf - lnKc);
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        const int sf = mk->rf[r][m], sb = mk->rr[r][m];
        fwd *= sf >= 0 ? sConc[max(sf, 0)][p] : 1.0;
        rev *= sb >= 0 ? sConc[max(sb, 0)][p] : 1.0;
      }
      return fwd - rev;
    };
    const int nitems = nr * NN;
    for (int idx = t; idx < nitems; idx += 2 * NTH) {
      const bool two = idx + NTH < nitems;
      // a wavefront none of whose lanes holds a second item forms one rate per lane
      const bool wave_two = (idx & ~63) + NTH < nitems;
      if (wave_two) {
        const int idx2 = two ? idx + NTH : idx;
        const double ra = rate(idx), rb = rate(idx2);
        sRate[idx / NN][idx % NN] = ra;
        if (two) sRate[idx2 / NN][idx2 % NN] = rb;
      } else {
        sRate[idx / NN][idx % NN] = rate(idx);
      }
    }
  }

  // 5. Rusanov total flux f = (g- + g+)/2 - lambda (w+ - w-)/2 at faces e0 + ff; at PE
  //    interfaces the synchronous flux is published and the AT combination is used
  //    (needs only the point phase: it runs beside the rates, from the last lane down, where
  //    lanes hold one rate item, not two)
  for (int idx = NTH - 1 - t; idx < V * (TE + 1); idx += NTH) {
    const int v = idx / (TE + 1), ff = idx % (TE + 1);
    const double wm = sTp[v][ff + 1], wp = sTm[v][ff + 2];
    const double lam = fmax(sLam[0][ff], sLam[1][ff]);
    const double diss = lam * (wp - wm);
    const int i = sI[ff + 1];
    double F;
    if (i >= 0) {
      const double Fs = 0.5 * (sGs[0][v][ff] + sGs[1][v][ff] - diss);
      if (ff < nloc && v < Vg) ring_at(a.ring, nmod, stage, a.dl.nif, i)[a.ring.off_F + v] = Fs;
      F = sK[ff + 1] > 0 ? sFat[v][ff] : Fs;
    } else {
      F = 0.5 * (sGf[0][v][ff] + sGf[1][v][ff] - diss);
    }
    sF[v][ff] = F;
  }
  __syncthreads();
  // species production W_i omega_i = W_i sum_r nu_ir (rate r), one lane per (node, species);
  // four terms per round trip (the entries past a species' count hold coefficient 0,
  // reaction 0, and add nothing)
  static_assert(kNsMaxReactions % 4 == 0, "species lists are read in fours");
  for (int idx = t; idx < NS * NN; idx += NTH) {
    const int i = idx / NN, p = idx % NN;
    double wdot = 0.0;
    const int cnt = mk->spn[i];
    for (int m0 = 0; m0 < cnt; m0 += 4) {
      double nu[4], rt[4];
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        nu[d] = (double)mk->spnu[i][m0 + d];
        rt[d] = sRate[mk->spr[i][m0 + d]][p];
      }
#pragma unroll
      for (int d = 0; d < 4; ++d) wdot += nu[d] * rt[d];
    }
    sS[i][p] = mk->W[i] * wdot;
  }
  __syncthreads();

  // 6. lift, source projection, SSP-RK3 combination
#pragma unroll
  for (int m = 0; m < kOut; ++m) {
    const int idx = t + m * NTH;
    if (idx >= V * M * TE) break;
    const int c = idx / TE, el = idx % TE;   // output component c of local element el
    if (el >= nloc || c >= VMg) continue;
    const int v = c / M, j = c % M;
    OpT vol = 0;
    double srcs = 0.0;
    const double gref = kMixed ? sG[v][el * Q] : 0.0;
#pragma unroll
    for (int qn = 0; qn < Q; ++qn) {
      if constexpr (kMixed) vol += (OpT)sWG[qn][j] * (OpT)(sG[v][el * Q + qn] - gref);
      else vol += (OpT)sWG[qn][j] * (OpT)sG[v][el * Q + qn];
      if (v >= 3) srcs += sWB[qn][j] * sS[v >= 3 ? v - 3 : 0][el * Q + qn];
    }
    const double src = srcs;
    const double half2j1 = 0.5 * (2 * j + 1);
    double b;
    if constexpr (kMixed) {
      // sum_q w_q P_j'(xi_q) gref = (1 - (-1)^j) gref, folded into the face terms
      const double fr = sF[v][el + 1] - gref, fl = sF[v][el] - gref;
      b = (double)vol - fr + ((j & 1) ? -fl : fl);
    } else {
      b = (double)vol - sF[v][el + 1] + ((j & 1) ? -sF[v][el] : sF[v][el]);
    }
    const double L = 2.0 * a.inv_dx * (half2j1 * b) + half2j1 * src;
    const size_t gi = sidx(e0 + el, c, VMg);
    double o;
    // explicit fused multiply-adds: the single-problem and batched kernels round alike
    if (rk.two_n) {
      const double kn = use_prev ? fma(rk.ca, w0pre[m], a.dt * L) : a.dt * L;
      kbuf[gi] = kn;
      o = fma(rk.cb, kn, sW[c][el + 2]);
    } else {
      const double y = fma(a.dt, L, sW[c][el + 2]);
      o = use_prev ? fma(rk.ca, w0pre[m], rk.cb * y) : y;
    }
    wout[gi] = o;
  }
  if (!ok) atomicOr(a.err, (int)kErrState);
  if (advance) advance_step(a.step, par, n, e0 == 0);
}

template <int M, int NS, int TE, int NTH, typename OpT>
__global__ __launch_bounds__(NTH) void ns_stage_kernel(NsArgs a) {
  __shared__ NsLds<M, NS, TE> L;
  __shared__ NsMechT<NS> smech;
  ns_tile<M, NS, OpT, NTH, TE>(a, a.ws, a.w0, a.wout, a.stage, a.advance, a.rk, a.kbuf,
                               xcd_item(blockIdx.x, gridDim.x) * TE, a.par, L, smech);
}

// LDS of the batched kernel: room for the largest order it serves, rates of up to
// kNsBatchReactions reactions.
template <int MMAX, int TE>
union NsBatchLds;
template <int TE>
union NsBatchLds<2, TE> {
  NsLds<2, kNsMaxSpecies, TE, kNsBatchReactions> m2;
};
template <int TE>
union NsBatchLds<3, TE> {
  NsLds<2, kNsMaxSpecies, TE, kNsBatchReactions> m2;
  NsLds<3, kNsMaxSpecies, TE, kNsBatchReactions> m3;
};
template <int TE>
union NsBatchLds<4, TE> {
  NsLds<2, kNsMaxSpecies, TE, kNsBatchReactions> m2;
  NsLds<3, kNsMaxSpecies, TE, kNsBatchReactions> m3;
  NsLds<4, kNsMaxSpecies, TE, kNsBatchReactions> m4;
};
template <int TE>
union NsBatchLds<5, TE> {
  NsLds<2, kNsMaxSpecies, TE, kNsBatchReactions> m2;
  NsLds<3, kNsMaxSpecies, TE, kNsBatchReactions> m3;
  NsLds<4, kNsMaxSpecies, TE, kNsBatchReactions> m4;
  NsLds<5, kNsMaxSpecies, TE, kNsBatchReactions> m5;
};

// Batched stage kernel: one workgroup per (instance, tile) entry of the work
// list; instances differ in size, order (up to MMAX modes), PE layout and
// delays, and all are at step counter parity par.  Sizing the LDS for the
// largest order present keeps more workgroups resident when the batch holds
// only low orders.  An instance whose step count has reached its target is
// skipped by all of its workgroups (its first tile carries the count over to
// the other parity at the last stage).
// At most 128 VGPRs (four wavefronts per SIMD): with four tiles' LDS per CU, more registers would
// leave only three of them resident (measured: 24 % slower at 132 VGPRs).  The LDS of tiles of up
// to N_p = 3 likewise stays within a quarter of the CU's 160 KiB.
static_assert(sizeof(NsBatchLds<4, 8>) + sizeof(NsMech) <= 40960, "four batched tiles of N_p <= 3 per CU");
template <typename OpT, int MMAX, int TE>
__global__ __launch_bounds__(kThreadsBatch, 4) void ns_batch_kernel(const NsArgs *__restrict__ insts,
                                                            const int2 *__restrict__ tiles, int stage, int par) {
  __shared__ NsBatchLds<MMAX, TE> L;
  __shared__ NsMech smech;
  const int2 tl = tiles[blockIdx.x];
  const NsArgs &a = insts[tl.x];
  const long long n = a.step[par];
  if (n >= a.target) {
    if (stage == 2 && tl.y == 0 && threadIdx.x == 0) a.step[par ^ 1] = n;
    return;
  }
  const int in_buf = stage, out_buf = stage == 2 ? 0 : stage + 1;
  const double *ws = a.W[in_buf];
  const double *w0 = a.W[0];
  double *wout = a.W[out_buf];
  const int M = a.M;
  const RkStage rk = rk_stage(ADG_SSPRK3, stage);   // batches run SSP-RK3
  constexpr int LP = kBatchLanesPerPoint, NR = kNsBatchReactions, NTH = kThreadsBatch;
  constexpr int NS = kNsMaxSpecies;
  if (M == 2) {
    ns_tile<2, NS, OpT, NTH, TE, LP, NR>(a, ws, w0, wout, stage, stage == 2, rk, nullptr, tl.y, par, L.m2, smech);
  } else if constexpr (MMAX >= 3) {
    if (M == 3) {
      ns_tile<3, NS, OpT, NTH, TE, LP, NR>(a, ws, w0, wout, stage, stage == 2, rk, nullptr, tl.y, par, L.m3, smech);
    } else if constexpr (MMAX >= 4) {
      if (M == 4) {
        ns_tile<4, NS, OpT, NTH, TE, LP, NR>(a, ws, w0, wout, stage, stage == 2, rk, nullptr, tl.y, par, L.m4, smech);
      } else if constexpr (MMAX >= 5) {
        // N_p = 4 keeps FP64 operators in a mixed batch: FP32 rounding would exceed a tenth of the
        // discretisation error there
        ns_tile<5, NS, double, NTH, TE, LP, NR>(a, ws, w0, wout, stage, stage == 2, rk, nullptr, tl.y, par, L.m5, smech);
      }
    }
  }
}

// ------------------------------------------------------------------ host side

bool ns_supported(int n_species, int n_reactions) {
  return n_species >= 1 && n_species <= kNsWideSpecies && n_reactions >= 1 && n_reactions <= kNsMaxReactions;
}

size_t ns_mech_bytes(int n_species) {
  return ns_capacity(n_species) == kNsMaxSpecies ? sizeof(NsMech) : sizeof(NsMechWide);
}

template <int NSC>
static adg_status upload_mech(const adg_physics *ph, void *dev_mech) {
  NsMechT<NSC> hm;
  const adg_status rc = ns_build_mech(ph, hm);
  if (rc != ADG_OK) return rc;
  if (hipMemcpy(dev_mech, &hm, sizeof hm, hipMemcpyHostToDevice) != hipSuccess) return ADG_ERR_HIP;
  return ADG_OK;
}

adg_status ns_setup(NsArgs &a, const adg_physics *ph, const adg_discretization *d, int E, int M, bool periodic,
                    double dx, const DelayParams &dl, const RingParams &rp, const Tables &tb, const int *face_if,
                    long long *step, int *err, void *dev_mech) {
  const int ns = ph->mech->n_species;
  const adg_status rc = ns_capacity(ns) == kNsMaxSpecies ? upload_mech<kNsMaxSpecies>(ph, dev_mech)
                                                         : upload_mech<kNsWideSpecies>(ph, dev_mech);
  if (rc != ADG_OK) return rc;
  a.ns = ns;
  a.periodic = periodic ? 1 : 0;
  a.at_in = nullptr;
  a.at_out = nullptr;
  a.nst = 3;
  a.face_if = face_if;
  a.step = step;
  a.err = err;
  a.mech = dev_mech;
  a.E = E;
  a.viscous = ph->viscous;
  a.dt = d->dt;
  a.inv_dx = 1.0 / dx;
  a.dl = dl;
  a.ring = rp;
  a.tb = tb;
  a.M = M;
  return ADG_OK;
}

template <int NSC>
adg_status ns_build_mech(const adg_physics *ph, NsMechT<NSC> &hm) {
  const adg_mechanism *m = ph->mech;
  if (!ns_supported(m->n_species, m->n_reactions) || m->n_species > NSC) return ADG_ERR_UNSUPPORTED;
  std::memset(&hm, 0, sizeof hm);
  // padded species: zero thermo, no reactions, unit molecular weight (finite 1/W)
  for (int i = m->n_species; i < NSC; ++i) hm.W[i] = hm.invW[i] = 1.0;
  hm.ns = m->n_species;
  hm.nr = m->n_reactions;
  hm.Ru = m->Ru;
  hm.p_ref = m->p_ref;
  hm.T_guess = m->T_guess;
  hm.mu_ref = m->mu_ref;
  hm.ln_T_ref = std::log(m->T_ref);
  hm.mu_exp = m->mu_exp;
  hm.inv_prandtl = 1.0 / m->prandtl;
  hm.ln_p_over_Ru = std::log(m->p_ref / m->Ru);
  for (int i = 0; i < hm.ns; ++i) {
    hm.W[i] = m->W[i];
    hm.invW[i] = 1.0 / m->W[i];
    hm.Ri[i] = m->Ru / m->W[i];
    const double *c = m->nasa7 + 7 * i;
    for (int k = 0; k < 7; ++k) hm.a[i][k] = c[k];
    hm.h2[i][0] = c[1] / 2.0;
    hm.h2[i][1] = c[2] / 3.0;
    hm.h2[i][2] = c[3] / 4.0;
    hm.h2[i][3] = c[4] / 5.0;
    hm.s2[i][0] = c[2] / 2.0;
    hm.s2[i][1] = c[3] / 3.0;
    hm.s2[i][2] = c[4] / 4.0;
    hm.ek[i][0] = hm.Ri[i] * (c[0] - 1.0);
    for (int q = 0; q < 4; ++q) hm.ek[i][1 + q] = hm.Ri[i] * hm.h2[i][q];
    hm.ek[i][5] = hm.Ri[i] * c[5];
    hm.ek[i][6] = hm.Ri[i];
    hm.ek[i][7] = 0.0;
  }
  for (int r = 0; r < hm.nr; ++r) {
    if (!(m->A[r] > 0.0)) return ADG_ERR_ARG;
    hm.lnA[r] = std::log(m->A[r]);
    hm.b[r] = m->b[r];
    hm.EaR[r] = m->Ea[r] / m->Ru;
    int dnu = 0;
    for (int i = 0; i < hm.ns; ++i) {
      const int f = m->nu_f[r * hm.ns + i], b = m->nu_r[r * hm.ns + i];
      if (f < 0 || f > 2 || b < 0 || b > 2) return ADG_ERR_UNSUPPORTED;
      dnu += b - f;
    }
    hm.dnu[r] = dnu;
    int nf = 0, nb = 0, g = 0;
    hm.rf[r][0] = hm.rf[r][1] = hm.rr[r][0] = hm.rr[r][1] = -1;
    for (int i = 0; i < hm.ns; ++i) {
      const int fi = m->nu_f[r * hm.ns + i], bi = m->nu_r[r * hm.ns + i];
      for (int c = 0; c < fi; ++c) {
        if (nf == 2) return ADG_ERR_UNSUPPORTED;   // at most two reactant molecules
        hm.rf[r][nf++] = i;
      }
      for (int c = 0; c < bi; ++c) {
        if (nb == 2) return ADG_ERR_UNSUPPORTED;
        hm.rr[r][nb++] = i;
      }
      const int nu = bi - fi;
      if (nu != 0) {
        hm.spr[i][hm.spn[i]] = (unsigned char)r;
        hm.spnu[i][hm.spn[i]] = (signed char)nu;
        hm.spn[i] += 1;
        if (g == 4) return ADG_ERR_UNSUPPORTED;
        hm.gidx[r][g] = i;
        hm.gnu[r][g] = nu;
        ++g;
      }
    }
  }
  return ADG_OK;
}

template <int M, int NS, int TE, int NTH, typename OpT>
static hipError_t ns_launch(const NsArgs &a, hipStream_t s) {
  const int blocks = (a.E + TE - 1) / TE;
  hipLaunchKernelGGL((ns_stage_kernel<M, NS, TE, NTH, OpT>), dim3(blocks), dim3(NTH), 0, s, a);
  return hipGetLastError();
}

template <int M, int NS, typename OpT>
static hipError_t ns_M(int cfg, const NsArgs &a, hipStream_t s) {
  switch (cfg) {
    case 0: return ns_launch<M, NS, 8, 512, OpT>(a, s);
    case 1: return ns_launch<M, NS, 8, 256, OpT>(a, s);
    case 2: return ns_launch<M, NS, 4, 256, OpT>(a, s);
    case 3: return ns_launch<M, NS, 4, 512, OpT>(a, s);
    case 4: return ns_launch<M, NS, 8, 1024, OpT>(a, s);
  }
  return hipErrorInvalidValue;
}

template <typename OpT, int TE>
static void batch_launch(int max_m, const NsArgs *insts, const int2 *tiles, int ntiles, int stage, int par,
                         hipStream_t s) {
  switch (max_m) {
    case 2: hipLaunchKernelGGL((ns_batch_kernel<OpT, 2, TE>), dim3(ntiles), dim3(kThreadsBatch), 0, s, insts, tiles, stage, par); break;
    case 3: hipLaunchKernelGGL((ns_batch_kernel<OpT, 3, TE>), dim3(ntiles), dim3(kThreadsBatch), 0, s, insts, tiles, stage, par); break;
    case 4: hipLaunchKernelGGL((ns_batch_kernel<OpT, 4, TE>), dim3(ntiles), dim3(kThreadsBatch), 0, s, insts, tiles, stage, par); break;
    default: hipLaunchKernelGGL((ns_batch_kernel<OpT, 5, TE>), dim3(ntiles), dim3(kThreadsBatch), 0, s, insts, tiles, stage, par); break;
  }
}

hipError_t launch_ns_batch(const NsArgs *insts, const int2 *tiles, int ntiles, int stage, int par, bool mixed,
                           int max_m, int tile_elems, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (max_m < 2 || max_m > kMaxM || (tile_elems != 4 && tile_elems != 8)) return hipErrorInvalidValue;
  if (tile_elems == 8) {
    if (mixed) batch_launch<float, 8>(max_m, insts, tiles, ntiles, stage, par, s);
    else batch_launch<double, 8>(max_m, insts, tiles, ntiles, stage, par, s);
  } else {
    if (mixed) batch_launch<float, 4>(max_m, insts, tiles, ntiles, stage, par, s);
    else batch_launch<double, 4>(max_m, insts, tiles, ntiles, stage, par, s);
  }
  return hipGetLastError();
}

template <int NS>
static hipError_t ns_stage_ns(int M, int cfg, const NsArgs &a, bool mixed, hipStream_t s) {
  // FP32 operators for N_p <= 3 only (N_p = 4 keeps FP64 ones: error budget)
  switch (M) {
    case 2: return mixed ? ns_M<2, NS, float>(cfg, a, s) : ns_M<2, NS, double>(cfg, a, s);
    case 3: return mixed ? ns_M<3, NS, float>(cfg, a, s) : ns_M<3, NS, double>(cfg, a, s);
    case 4: return mixed ? ns_M<4, NS, float>(cfg, a, s) : ns_M<4, NS, double>(cfg, a, s);
    case 5: return ns_M<5, NS, double>(cfg, a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_ns_stage(int M, int cfg, const NsArgs &a, bool mixed, hipStream_t s) {
  return ns_capacity(a.ns) == kNsMaxSpecies ? ns_stage_ns<kNsMaxSpecies>(M, cfg, a, mixed, s)
                                            : ns_stage_ns<kNsWideSpecies>(M, cfg, a, mixed, s);
}

template adg_status ns_build_mech<kNsMaxSpecies>(const adg_physics *, NsMech &);
template adg_status ns_build_mech<kNsWideSpecies>(const adg_physics *, NsMechWide &);

}  // namespace adg
