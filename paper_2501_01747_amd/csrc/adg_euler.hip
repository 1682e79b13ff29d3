// Stage kernel of the one-step reactive Euler model, with the troubled-cell
// indicator and the characteristic (AT-)WENO limiter of a limited problem in the
// same kernel.
//
// Stage (Sec. 3.1 Eq. (5), Sec. 3.2 Eq. (7)): one thread per element; each
// wavefront owns 62 consecutive elements (60 with the limiter) and holds one
// neighbour (two with the limiter) on each side.  Every lane loads its element's
// modal DoFs from the component planes (coalesced) and forms both face traces;
// one numerical flux per face is computed and passed to the neighbouring lane by
// a shuffle; at PE-interface faces the synchronous flux of this level is written
// to the history ring and replaced by the AT combination of past levels.  The
// volume integral, the source projection, the lift and the RK combination then
// run in registers and the output is stored once.
//
// Limiter (Sec. 3.3, Eq. (9)-(11)): with a second halo lane on each side, every
// owned element's two neighbours have their unlimited stage outputs inside the
// same wavefront, so the indicator and the WENO reconstruction read them from
// LDS; no other wavefront's output is needed, and the limited values are stored
// in place of the unlimited ones with no further pass (every stencil still sees
// unlimited data, the simultaneous application of the limiter).  HBM traffic per
// stage: read w^(s) (+ w^n for stages 2 and 3), write w^(s+1), plus a flag byte
// per element with the limiter.
#include "adg_device.hpp"

namespace adg {

template <int M>
__device__ __forceinline__ void traces(const double (&u)[5][M], double *wl, double *wr) {
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    double sm = 0.0, sp = 0.0;
#pragma unroll
    for (int j = 0; j < M; ++j) {
      sp += u[v][j];
      sm += (j & 1) ? -u[v][j] : u[v][j];
    }
    wl[v] = sm;
    wr[v] = sp;
  }
}

template <int M>
__device__ __forceinline__ void load_elem(const double *__restrict__ w, int E, int e, double (&u)[5][M]) {
#pragma unroll
  for (int v = 0; v < 5; ++v)
#pragma unroll
    for (int j = 0; j < M; ++j) u[v][j] = w[sidx(e, v * M + j, 5 * M)];
}

// The AT flux of Eq. (7) at PE interface i with delay k > 0: the past levels' synchronous
// fluxes of this stage combined with the Eq. (8) weights.  Levels 0..3 are loaded together
// (a level past q reads level n-k with weight 0), later ones (q > 4) one at a time.
__device__ __forceinline__ void at_flux(const EulerArgs &a, int nmod, int i, int k, double (&acc)[5]) {
#pragma unroll
  for (int v = 0; v < 5; ++v) acc[v] = 0.0;
  const int q = a.dl.q;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const bool in = j < q;
    const double c = in ? at_weight(q, k, j) : 0.0;
    const double *h = ring_at(a.ring, ring_slot(nmod, k + (in ? j : 0), a.ring.D), a.stage, a.dl.nif, i) + a.ring.off_F;
#pragma unroll
    for (int v = 0; v < 5; ++v) acc[v] += c * h[v];
  }
  for (int j = 4; j < q; ++j) {
    const double c = at_weight(q, k, j);
    const double *h = ring_at(a.ring, ring_slot(nmod, k + j, a.ring.D), a.stage, a.dl.nif, i) + a.ring.off_F;
#pragma unroll
    for (int v = 0; v < 5; ++v) acc[v] += c * h[v];
  }
}

// Numerical flux at a face from its two traces; at PE interface i the synchronous flux
// is published for this level and, with delay k > 0, replaced by the AT flux Fat.
template <int FLUX>
__device__ __forceinline__ bool face_flux(const EulerArgs &a, int nmod, int i, int k, const double (&Fat)[5],
                                          const double *wm, const double *wp, double *F) {
  bool ok = numflux1<FLUX>(a.ph, wm, wp, F);
  if (i >= 0) {
    double *rec = ring_at(a.ring, nmod, a.stage, a.dl.nif, i) + a.ring.off_F;
#pragma unroll
    for (int v = 0; v < 5; ++v) rec[v] = F[v];
    if (k > 0) {
#pragma unroll
      for (int v = 0; v < 5; ++v) F[v] = Fat[v];
    }
  }
  return ok;
}

// ------------------------------------------------------------------- limiter

// Characteristic left and right eigenvectors at the mean state (one-step model).
// Rows of L (linear forms in the conserved variables):
//   (dp - rho a du)/(2a^2), drho - dp/a^2, d(rho Y_R) - Y_R drho,
//   d(rho Y_R + rho Y_P - rho), (dp + rho a du)/(2a^2),
// with dp and du the differentials of p and u.  R = L^-1 in closed form: column k
// is the conserved perturbation whose characteristic variables are e_k, built from
// the primitive perturbations (drho, du, dp, dY_R) that L maps to e_k.  L involves
// Y_R only, so the product entry of the columns with drho = 1 is 1 - Y_R (not the
// mean state's Y_P): R is then the exact inverse for any state, and the limiter
// keeps rho Y_R + rho Y_P - rho at round-off instead of feeding its round-off back.
// Field c only: row c of L into lr, column c of R into rc.
__device__ __forceinline__ bool char_row_col(const OneStep &ph, const double *wb, int c, double (&lr)[5],
                                             double (&rc)[5]) {
  Prim1 pr;
  const bool ok = prim1(ph, wb, pr);
  const double rho = pr.rho, u = pr.u, a = pr.a, g1 = ph.gamma - 1.0, q = ph.q_heat;
  const double irho = 1.0 / rho;
  const double dp[5] = {g1 * 0.5 * u * u, -g1 * u, g1, -g1 * q, 0.0};
  const double du[5] = {-u * irho, irho, 0.0, 0.0, 0.0};
  const double a2 = a * a, ia2 = 1.0 / a2;
  const double YR = wb[3] * irho, YP = 1.0 - YR;
  const double l2[5] = {-YR, 0.0, 0.0, 1.0, 0.0};
  const double l3[5] = {-1.0, 0.0, 0.0, 1.0, 1.0};
  // the acoustic rows carry the sign of their wave speed u -+ a
  const double sa = c == 0 ? -1.0 : 1.0;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const double drho = k == 0 ? 1.0 : 0.0;
    const double ac = (dp[k] + sa * rho * a * du[k]) * (0.5 * ia2);
    lr[k] = (c == 0 || c == 4) ? ac : c == 1 ? drho - dp[k] * ia2 : c == 2 ? l2[k] : l3[k];
  }
  // columns: acoustic -, entropy, reactant, species sum, acoustic +
  const double hk = 0.5 * u * u + q * YR;   // d(rho E)/d rho at fixed u, p, Y
  const double ha = a2 / g1;
  if (c == 0 || c == 4) {
    rc[0] = 1.0; rc[1] = u + sa * a; rc[2] = ha + hk + sa * u * a; rc[3] = YR; rc[4] = YP;
  } else if (c == 1) {
    rc[0] = 1.0; rc[1] = u; rc[2] = hk; rc[3] = YR; rc[4] = YP;
  } else if (c == 2) {
    rc[0] = 0.0; rc[1] = 0.0; rc[2] = q; rc[3] = 1.0; rc[4] = -1.0;
  } else {
    rc[0] = 0.0; rc[1] = 0.0; rc[2] = 0.0; rc[3] = 0.0; rc[4] = 1.0;
  }
  return ok && a > 0.0;
}

// minmod of three numbers: the one of least magnitude if all share a sign, else 0
__device__ __forceinline__ double minmod3(double x, double y, double z) {
  if (x > 0.0 && y > 0.0 && z > 0.0) return fmin(x, fmin(y, z));
  if (x < 0.0 && y < 0.0 && z < 0.0) return fmax(x, fmax(y, z));
  return 0.0;
}

template <int M>
__device__ __forceinline__ double trace_at(const double (&c)[M], int side) {
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < M; ++j) s += (side == 0 && (j & 1)) ? -c[j] : c[j];
  return s;
}

// Where the limiter of an owned element takes the neighbour across one face from:
// LDS at base + v sv + j sj.  Either the neighbouring lane's unlimited output, or one
// of the wavefront's slots holding, at a transmissive end (ghost), the constant equal
// to the element's own mean, or at a PE interface i with effective delay k > 0 the
// Eq. (11) AT combination of the unlimited outputs that past levels published to the
// history ring, formed once per stage.
struct NbSide {
  int base, sv, sj, i, k, ghost;
};

// LDS per wavefront: the unlimited outputs [5M][64], then kNbSlots neighbours [5M]:
// two per lane for kSlotLanes lanes at a time.
constexpr int kSlotLanes = 4;
constexpr int kNbSlots = 2 * kSlotLanes;
template <int M>
constexpr int lds_wave_doubles() { return 5 * M * 64 + kNbSlots * 5 * M; }

// The Eq. (11) combination of the modal data of the neighbour across PE interface i
// with delay k (side 0: the element left of it, the first U block of the record),
// variable by variable in c[5M].
template <int M>
__device__ __forceinline__ void at_neighbour(const EulerArgs &a, long long n, int nmod, int i, int k, int side,
                                             double (&c)[5 * M]) {
#pragma unroll
  for (int t = 0; t < 5 * M; ++t) c[t] = 0.0;
  const int off = a.ring.off_U + (side == 0 ? 0 : 5 * M);
  // two levels per round trip (a level past q reads level n-k with weight 0); mode j of the
  // hybrid stencil takes weight 0 past its own max(1, q - j) levels
  for (int j0 = 0; j0 < a.dl.q; j0 += 2) {
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      const int jj = j0 + d;
      const bool in = jj < a.dl.q;
      double w[M];
#pragma unroll
      for (int m = 0; m < M; ++m) w[m] = in ? buffer_weight(a.dl, k, m, jj) : 0.0;
      const double *h = ring_at(a.ring, ring_slot(nmod, k + (in ? jj : 0), a.ring.D), a.stage, a.dl.nif, i) + off;
#pragma unroll
      for (int t = 0; t < 5 * M; ++t) c[t] += w[t % M] * h[t];
    }
  }
}

// Modes of variable v of the neighbour across one face.  ls is the wavefront's LDS area.
template <int M>
__device__ __forceinline__ void nb_var(const NbSide &sd, int v, const double *ls, double (&c)[M]) {
#pragma unroll
  for (int j = 0; j < M; ++j) c[j] = ls[sd.base + v * sd.sv + j * sd.sj];
}

// Troubled-cell indicator of an owned element with unlimited modes u (KXRCF or TVB
// minmod).
template <int M>
__device__ __forceinline__ bool troubled(const EulerArgs &a, const LimiterArgs &l, int nmod,
                                         const NbSide (&sd)[2], const double (&u)[5][M], const double *ls,
                                         int lane) {
  const bool ghostL = sd[0].ghost, ghostR = sd[1].ghost;
  bool flag = false;
  if (l.indicator == 2) {
    flag = true;   // every cell limited (the accuracy-test setting of the WENO limiter)
  } else if (l.indicator == 1) {
    // TVB minmod: the face deviations from the mean against the mean differences, every
    // variable; differences within 1e-10 of the largest |mean| of any variable in the
    // stencil count as equal (round-off in a constant state is not a slope)
    double mL[5], mR[5];
    double scale = 0.0;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      double c[M];
      nb_var<M>(sd[0], v, ls, c);
      mL[v] = c[0];
      nb_var<M>(sd[1], v, ls, c);
      mR[v] = c[0];
      scale = fmax(scale, fmax(fabs(u[v][0]), fmax(fabs(mL[v]), fabs(mR[v]))));
    }
    const double tol = 1e-10 * scale;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const double m = u[v][0];
      const double dp = trace_at<M>(u[v], 1) - m, dm = m - trace_at<M>(u[v], 0);
      const double Dp = mR[v] - m, Dm = m - mL[v];
      const double mp = fabs(dp) <= l.tvb_mh2 ? dp : minmod3(dp, Dp, Dm);
      const double mm = fabs(dm) <= l.tvb_mh2 ? dm : minmod3(dm, Dp, Dm);
      if (fabs(mp - dp) > tol || fabs(mm - dm) > tol) flag = true;
    }
  } else {
    // KXRCF: jumps at inflow faces against h^((N_p+1)/2) max_q |w(xi_q)|, on rho and rho E;
    // tL/tR: the neighbours' traces at the shared faces of rho, rho u, rho E
    double tL[3], tR[3];
#pragma unroll
    for (int v = 0; v < 3; ++v) {
      double c[M];
      nb_var<M>(sd[0], v, ls, c);
      tL[v] = trace_at<M>(c, 1);
      nb_var<M>(sd[1], v, ls, c);
      tR[v] = trace_at<M>(c, 0);
    }
    const double uL_e = trace_at<M>(u[1], 0) / trace_at<M>(u[0], 0);
    const double uR_e = trace_at<M>(u[1], 1) / trace_at<M>(u[0], 1);
    const double uL_n = ghostL ? uL_e : tL[1] / tL[0];
    const double uR_n = ghostR ? uR_e : tR[1] / tR[0];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int v = t == 0 ? 0 : 2;
      double jump = 0.0;
      if (0.5 * (uL_e + uL_n) > 0.0 && !ghostL) jump += trace_at<M>(u[v], 0) - tL[v];
      if (0.5 * (uR_e + uR_n) < 0.0 && !ghostR) jump += trace_at<M>(u[v], 1) - tR[v];
      double norm = 0.0;
#pragma unroll
      for (int q = 0; q < M; ++q) {
        double val = 0.0;
#pragma unroll
        for (int j = 0; j < M; ++j) val += u[v][j] * a.tb.B[q][j];
        norm = fmax(norm, fabs(val));
      }
      if (fabs(jump) / (l.kx_h * norm) > 1.0) flag = true;
    }
  }
  return flag;
}

// The simple WENO reconstruction of Eq. (9)-(10) of one characteristic field with
// modes vc in the cell and vL, vR in its neighbours: the limited modes vl.
template <int M>
__device__ __forceinline__ void weno_field(const LimiterArgs &l, const double (&vc)[M], const double (&vL)[M],
                                           const double (&vR)[M], double (&vl)[M]) {
  // re-expand the neighbours in the cell's coordinate and reset their mean
  double tL[M], tR[M];
#pragma unroll
  for (int k2 = 0; k2 < M; ++k2) {
    double sl = 0.0, sr = 0.0;
#pragma unroll
    for (int j = 0; j < M; ++j) {
      sl += l.Tl[k2][j] * vL[j];
      sr += l.Tr[k2][j] * vR[j];
    }
    tL[k2] = sl; tR[k2] = sr;
  }
  tL[0] = vc[0];
  tR[0] = vc[0];
  double beta[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int p = 0; p < M; ++p)
#pragma unroll
    for (int r = 0; r < M; ++r) {
      beta[0] += tL[p] * l.Bm[p][r] * tL[r];
      beta[1] += vc[p] * l.Bm[p][r] * vc[r];
      beta[2] += tR[p] * l.Bm[p][r] * tR[r];
    }
  double wbar[3], sum = 0.0;
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const double d = l.eps + beta[s];
    wbar[s] = l.gam[s] / (d * d);
    sum += wbar[s];
  }
  const double isum = 1.0 / sum;
  const double om0 = wbar[0] * isum, om1 = wbar[1] * isum, om2 = wbar[2] * isum;
#pragma unroll
  for (int j = 0; j < M; ++j) vl[j] = om0 * tL[j] + om1 * vc[j] + om2 * tR[j];
}

// Characteristic WENO of the troubled element x_c whose unlimited modes sit in lane cl
// of the wavefront's LDS area, by a group of 8 lanes: lane c < 5 limits characteristic
// field c (lanes 5..7 repeat field 4 and contribute nothing); w_lim[v] = sum_c R[v][c]
// v_c^lim is summed across the group in a fixed butterfly order and lane v writes
// variable v.  Returns false if the mean state has no valid characteristic decomposition.
template <int M>
__device__ __forceinline__ bool weno_group(const EulerArgs &a, const LimiterArgs &l, int nmod,
                                           const NbSide (&sd)[2], const double *ls, int cl, int c, double *wout,
                                           int xc) {
  double wb[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) wb[v] = ls[(v * M) * 64 + cl];
  double lr[5], rc[5];
  const bool ok = char_row_col(a.ph, wb, c < 5 ? c : 4, lr, rc);
  double vc[M], vL[M], vR[M];
#pragma unroll
  for (int j = 0; j < M; ++j) {
    vc[j] = 0.0; vL[j] = 0.0; vR[j] = 0.0;
  }
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    double cl_[M], cr_[M];
    nb_var<M>(sd[0], v, ls, cl_);
    nb_var<M>(sd[1], v, ls, cr_);
#pragma unroll
    for (int j = 0; j < M; ++j) {
      vc[j] += lr[v] * ls[(v * M + j) * 64 + cl];
      vL[j] += lr[v] * cl_[j];
      vR[j] += lr[v] * cr_[j];
    }
    // one variable's reads at a time: keeps the stage kernel's register budget
    __builtin_amdgcn_sched_barrier(0);
  }
  double vl[M];
  weno_field<M>(l, vc, vL, vR, vl);
#pragma unroll
  for (int v = 0; v < 5; ++v)
#pragma unroll
    for (int j = 0; j < M; ++j) {
      double part = c < 5 ? rc[v] * vl[j] : 0.0;
      part += dpp_move<kDppXor1>(part);
      part += dpp_move<kDppXor2>(part);
      part += dpp_move<kDppHalfMirror>(part);   // the same sum as from lane ^ 4
      if (c == v) wout[sidx(xc, v * M + j, 5 * M)] = part;
    }
  return ok;
}

// Slots of a wavefront's round (kSlotLanes elements, two slots each): the ghost or AT
// neighbour of every face of the element that needs one (AT slots only unless at_ready:
// the first round's are gathered at the start of the kernel), then the face's source
// points at its slot.  One pass over each element's first such face, a second over
// elements whose both faces need one.
template <int M>
__device__ __forceinline__ void fill_slots(const EulerArgs &a, long long n, int nmod, NbSide (&sd)[2], bool mine,
                                           int rank, double *ls, int lane, bool at_ready) {
  const bool need0 = sd[0].ghost || sd[0].k > 0, need1 = sd[1].ghost || sd[1].k > 0;
  const bool two = mine && need0 && need1;
#pragma unroll 1
  for (int pass = 0; pass < 2; ++pass) {
    const bool go = pass == 0 ? mine : two;
    if (!__ballot(go)) break;
    if (go) {
      const int side = (pass == 0 && need0) ? 0 : 1;
      const int slot = 2 * (rank % kSlotLanes) + side;
      double *sl = ls + 5 * M * 64 + slot * 5 * M;
      if (side == 0 ? sd[0].ghost : sd[1].ghost) {
#pragma unroll
        for (int v = 0; v < 5; ++v)
#pragma unroll
          for (int j = 0; j < M; ++j) sl[v * M + j] = j == 0 ? ls[(v * M) * 64 + lane] : 0.0;
      } else if (!at_ready) {
        double c[5 * M];
        at_neighbour<M>(a, n, nmod, side == 0 ? sd[0].i : sd[1].i, side == 0 ? sd[0].k : sd[1].k, side, c);
#pragma unroll
        for (int t = 0; t < 5 * M; ++t) sl[t] = c[t];
      }
      NbSide &t = side == 0 ? sd[0] : sd[1];
      t.base = 5 * M * 64 + slot * 5 * M;
      t.sv = M;
      t.sj = 1;
    }
  }
}

// The AT neighbours of a wavefront's first round (slot 2r + side belongs to the r-th lane
// of the wavefront that needs a slot), gathered by all lanes of the wavefront at once:
// lane l forms components l, l + 64, l + 128 of the slots' 8 x 5M, each the same Eq. (11)
// combination at_neighbour forms (levels in the same order, so the same rounding).
// Ghost slots are left to their owners.
template <int M>
__device__ __forceinline__ void gather_first_slots(const EulerArgs &a, int nmod, const NbSide (&sd)[2],
                                                   unsigned long long nball, double *ls, int lane) {
  constexpr int C = 5 * M;
#pragma unroll
  for (int q0 = 0; q0 < kNbSlots * C; q0 += 64) {
    const int pair = q0 + lane;
    const int s = min(pair / C, kNbSlots - 1), comp = pair % C;
    const int r = s >> 1, side = s & 1;
    unsigned long long m = nball;
    for (int j = 0; j < r; ++j) m &= m - 1;   // drop the r lowest lanes that need a slot
    const int src = m ? __ffsll((long long)m) - 1 : 0;
    const int i0 = __shfl(sd[0].i, src), i1 = __shfl(sd[1].i, src);
    const int k0 = __shfl(sd[0].k, src), k1 = __shfl(sd[1].k, src);
    const int i = side ? i1 : i0, k = side ? k1 : k0;   // a ghost side has i = -1, k = 0
    if (pair < kNbSlots * C && m != 0 && i >= 0 && k > 0) {
      const int off = a.ring.off_U + (side == 0 ? 0 : C) + comp;
      const int mode = comp % M;
      const int qm = buffer_levels(a.dl, mode);   // levels this mode uses (q, or max(1, q - mode))
      double acc = 0.0;
      // levels past qm read level n-k (no further load) with weight 0
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const bool in = j < qm;
        const double w = in ? buffer_weight(a.dl, k, mode, j) : 0.0;
        acc += w * ring_at(a.ring, ring_slot(nmod, k + (in ? j : 0), a.ring.D), a.stage, a.dl.nif, i)[off];
      }
      for (int j = 4; j < qm; ++j)
        acc += buffer_weight(a.dl, k, mode, j) *
               ring_at(a.ring, ring_slot(nmod, k + j, a.ring.D), a.stage, a.dl.nif, i)[off];
      ls[5 * M * 64 + s * C + comp] = acc;
    }
  }
}

// ---------------------------------------------------------------- stage kernel

// Wavefront-local stage kernel.  Lane l of a wavefront holds element
// base + l - H (base = (64 - 2H) * wavefront index, H = 1, or 2 with the
// limiter): lanes H .. 63-H own their element, the H lanes on each side hold
// neighbours, loaded together with the owned elements.  Lane k computes the flux
// at the face between its element and lane k+1's; traces and fluxes move between
// lanes by cross-lane shuffles.  With the limiter, lanes 1 and 62 also form their
// element's unlimited output (bitwise the value its owner forms), the wavefront
// stages its outputs in LDS (ls, 5M x 64 doubles per wavefront), and each owned
// element runs the indicator and, if troubled, the WENO reconstruction from them.
template <int M, int FLUX, bool LIM>
__device__ __forceinline__ void euler_stage_body(const EulerArgs &a, const LimiterArgs &l, double *lds, int *rounds,
                                                 int blk, int par) {
  constexpr int V = 5, Q = M;
  constexpr int H = LIM ? 2 : 1;
  constexpr int WE = 64 - 2 * H;
  const int lane = threadIdx.x & 63;
  const int base = ((blk * kEulerBlock + threadIdx.x) >> 6) * WE;
  const int E = a.E;
  const int xu = base + lane - H;                       // element index before periodic wrap
  const bool live = base < E;
  const bool own = live && lane >= H && lane < 64 - H && xu < E;
  const bool ghost_l = !a.periodic && xu == -1;         // transmissive ends: ghost = interior trace
  const bool ghost_r = !a.periodic && xu == E;
  // loaded: owned elements and H neighbours on each side (wrapped), never past a transmissive end
  const bool loads = live && (a.periodic ? xu <= E - 1 + H : (xu >= 0 && xu < E));
  // forms an output: owned, and with the limiter the first neighbour on each side
  const bool calc = LIM ? live && lane >= 1 && lane <= 62 && (a.periodic ? xu <= E : (xu >= 0 && xu < E)) : own;
  // computes the flux at face xu + 1 (faces 0..E; periodic faces wrap)
  const bool face_lane = live && lane <= 62 && (a.periodic ? xu + 1 <= E - 1 + H : (xu >= -1 && xu < E));
  int x = xu;   // within a few periods of [0, E)
  while (x < 0) x += E;
  while (x >= E) x -= E;
  int fidx = xu + 1;
  if (a.periodic && (fidx < 0 || fidx > E)) fidx = fidx < 0 ? fidx + E : fidx - E;
  // the PE interface at this lane's face: loaded first, beside the step counter (the
  // state's buffers and the delays depend on the step, the interface map does not)
  const int iface = face_lane ? a.face_if[fidx] : -1;
  const long long n = a.step[par];
  const int nmod = step_mod(n, a.ring.D);
  bool ok = true;
  const double *w0 = a.w0, *ws = a.ws;
  double *wout = a.wout;
  if (LIM && a.alt) {
    const int c = (int)(n & 1);
    w0 = a.W[c];
    ws = a.stage == 0 ? a.W[c] : a.stage == 1 ? a.W[1 - c] : a.W[2];
    wout = a.stage == 1 ? a.W[2] : a.W[1 - c];
  }

  double u[V][M], wn[V][M];
  // the second operand of the RK combination (w^n, or the 2N register) is loaded
  // together with the stage input, so both loads are in flight at once.  Without the
  // limiter only the owning lane reads an element, so the last Shu-Osher stage may
  // overwrite w^n and a 2N stage its register in place; the limiter's halo lanes read
  // other wavefronts' elements, so there every stage writes buffers it does not read.
  const bool use_prev = calc && (a.rk.two_n ? a.rk.ca != 0.0 : a.rk.ca != 0.0 || a.rk.cb != 1.0);
  if (use_prev) load_elem<M>(a.rk.two_n ? a.kbuf : w0, E, x, wn);
  if (loads) {
    load_elem<M>(ws, E, x, u);
  } else {
#pragma unroll
    for (int v = 0; v < V; ++v)
#pragma unroll
      for (int j = 0; j < M; ++j) u[v][j] = 0.0;
  }
  // a delayed PE-interface face gathers its past levels' fluxes now, while the state
  // loads are in flight
  // (the limiter kernel draws with the branch-free count, measured 0.9 us faster per stage on
  // the shock workload; the plain kernel with the ordered search, 0.6 us faster on the smooth one)
  const int kf = iface >= 0 ? eff_delay<LIM>(a.dl, n, iface) : 0;
  double Fat[V];
  if (kf > 0) at_flux(a, nmod, iface, kf, Fat);

  // with the limiter: this wavefront's outputs, [component][lane], and the neighbour
  // sources of the owned elements.  Faces at a transmissive end or a delayed PE interface
  // need a slot: kSlotLanes such elements per round, two slots each; the first round's AT
  // neighbours are gathered now, while the state loads are in flight.
  double *ls = LIM ? lds + (threadIdx.x >> 6) * lds_wave_doubles<M>() : nullptr;
  NbSide sd[2];
  bool needs = false;
  unsigned long long nball = 0;
  if constexpr (LIM) {
    // an owned element's faces x and x + 1 are the faces of the previous lane and of this one
    const int iface_prev = dpp_move<kDppFromPrev>(iface);
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const bool ghost = own && !a.periodic && (side == 0 ? x == 0 : x == E - 1);
      const int i = (own && !ghost) ? (side == 0 ? iface_prev : iface) : -1;
      const int k = i >= 0 ? eff_delay<true>(a.dl, n, i) : 0;
      sd[side].base = lane + (side == 0 ? -1 : 1);
      sd[side].sv = M * 64;
      sd[side].sj = 64;
      sd[side].i = i;
      sd[side].k = k;
      sd[side].ghost = ghost;
      needs = needs || ghost || k > 0;
    }
    nball = __ballot(needs);
    gather_first_slots<M>(a, nmod, sd, nball, ls, lane);
  }

  double wl[V], wr[V];
  traces<M>(u, wl, wr);
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const double next_l = dpp_move<kDppFromNext>(wl[v]);
    const double prev_r = dpp_move<kDppFromPrev>(wr[v]);
    if (ghost_l) wr[v] = next_l;
    if (ghost_r) wl[v] = prev_r;
  }
  // flux at the face to the right of this lane's element
  double F[V];
  {
    double wp[V];
#pragma unroll
    for (int v = 0; v < V; ++v) wp[v] = dpp_move<kDppFromNext>(wl[v]);
    const bool fok = face_flux<FLUX>(a, nmod, iface, kf, Fat, wr, wp, F);
    if (face_lane) ok = fok && ok;
  }
  double Fl[V];
#pragma unroll
  for (int v = 0; v < V; ++v) Fl[v] = dpp_move<kDppFromPrev>(F[v]);
  const int if_left = dpp_move<kDppFromPrev>(iface);

  if (calc) {
    // b_j = sum_q w_q P_j'(xi_q) f_q - F_{e+1} P_j(1) + F_e P_j(-1); the face terms go in first
    double vol[V][M], srcR[M];
#pragma unroll
    for (int j = 0; j < M; ++j) {
      srcR[j] = 0.0;
#pragma unroll
      for (int v = 0; v < V; ++v) vol[v][j] = -F[v] + ((j & 1) ? -Fl[v] : Fl[v]);
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      double wq[V];
#pragma unroll
      for (int v = 0; v < V; ++v) {
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < M; ++j) acc += u[v][j] * a.tb.B[q][j];
        wq[v] = acc;
      }
      Prim1 pr;
      ok = prim1(a.ph, wq, pr) && ok;
      double f[V];
      flux1(wq, pr, f);
      const double rate = a.ph.k_pre * wq[3] * exp(-a.ph.e_act * (pr.rho / pr.p));
#pragma unroll
      for (int j = 0; j < M; ++j) {
        const double g = a.tb.WG[q][j];
#pragma unroll
        for (int v = 0; v < V; ++v) vol[v][j] += g * f[v];
        srcR[j] += a.tb.WB[q][j] * (-rate);
      }
    }
    double *recR = (own && a.store_U && if_left >= 0)   // this element is right of interface if_left
                       ? ring_at(a.ring, nmod, a.stage, a.dl.nif, if_left) + a.ring.off_U + V * M : nullptr;
    double *recL = (own && a.store_U && iface >= 0)     // left of interface iface
                       ? ring_at(a.ring, nmod, a.stage, a.dl.nif, iface) + a.ring.off_U : nullptr;
#pragma unroll
    for (int v = 0; v < V; ++v) {
#pragma unroll
      for (int j = 0; j < M; ++j) {
        const double half2j1 = 0.5 * (2 * j + 1);
        double s = 0.0;
        if (v == 3) s = srcR[j];
        if (v == 4) s = -srcR[j];
        const double L = a.two_over_dx * (half2j1 * vol[v][j]) + half2j1 * s;
        const size_t gi = sidx(x, v * M + j, V * M);
        double o;
        // explicit fused multiply-adds: every kernel that runs this combination (single
        // problem or batch) rounds it the same way
        if (a.rk.two_n) {
          const double kn = use_prev ? fma(a.rk.ca, wn[v][j], a.dt * L) : a.dt * L;
          if (own) a.kout[gi] = kn;
          o = fma(a.rk.cb, kn, u[v][j]);
        } else {
          const double y = fma(a.dt, L, u[v][j]);
          o = use_prev ? fma(a.rk.ca, wn[v][j], a.rk.cb * y) : y;
        }
        if (LIM) ls[(v * M + j) * 64 + lane] = o;   // stored below, limited if troubled
        else if (own) wout[gi] = o;
        if (recR) recR[v * M + j] = o;
        if (recL) recL[v * M + j] = o;
      }
    }
  }

  if constexpr (LIM) {
    const int rank = __popcll(nball & ((1ull << lane) - 1ull));
    const int my_round = needs ? rank / kSlotLanes : 0;
    // the first round's ghost slots and slot pointers are set before the barrier: they need
    // only this lane's data (its AT slots were gathered at the start)
    fill_slots<M>(a, n, nmod, sd, needs && my_round == 0, rank, ls, lane, true);
    if (lane == 0) rounds[threadIdx.x >> 6] = (__popcll(nball) + kSlotLanes - 1) / kSlotLanes;
    __syncthreads();   // the wavefront's outputs and slots are in LDS; every wavefront's round count too
    int nrounds = 1;
#pragma unroll
    for (int w = 0; w < kEulerBlock / 64; ++w) nrounds = max(nrounds, rounds[w]);
#pragma unroll 1
    for (int round = 0; round < nrounds; ++round) {
      if (round > 0) {
        __syncthreads();   // the previous round's slots have been read
        fill_slots<M>(a, n, nmod, sd, needs && my_round == round, rank, ls, lane, false);
        __syncthreads();   // the slots are read by other lanes of the wavefront below
      }
      bool flag = false;
      if (own && my_round == round) {
        double u2[V][M];
#pragma unroll
        for (int v = 0; v < V; ++v)
#pragma unroll
          for (int j = 0; j < M; ++j) u2[v][j] = ls[(v * M + j) * 64 + lane];
        flag = troubled<M>(a, l, nmod, sd, u2, ls, lane);
        l.flags[x] = flag ? 1 : 0;
        if (flag) {
          atomicAdd(l.flag_count, 1ull);
        } else {
          // a rolled loop: the compiler would otherwise keep one 64-bit address per
          // component live across the limiter (and spill them)
          double *dst = wout + sidx(x, 0, V * M);
#pragma unroll 1
          for (int c = 0; c < V * M; ++c) dst[c * kLayoutBlock] = ls[c * 64 + lane];
        }
      }
      // troubled elements: eight at a time, one group of 8 lanes each (group g takes the
      // g-th lowest remaining troubled lane)
      unsigned long long rem = __ballot(flag);
      const int grp = lane >> 3, cf = lane & 7;
#pragma unroll 1
      while (rem) {
        unsigned long long r = rem;
        for (int g = 0; g < grp && r; ++g) r &= r - 1;
        const int cl = r ? __ffsll((long long)r) - 1 : -1;
        for (int g = 0; g < 8 && rem; ++g) rem &= rem - 1;
        const int src = cl < 0 ? 0 : cl;
        const int xc = __shfl(x, src);
        NbSide sc[2];
#pragma unroll
        for (int side = 0; side < 2; ++side) {
          sc[side].base = __shfl(sd[side].base, src);
          sc[side].sv = __shfl(sd[side].sv, src);
          sc[side].sj = __shfl(sd[side].sj, src);
          sc[side].i = __shfl(sd[side].i, src);
          sc[side].k = __shfl(sd[side].k, src);
          sc[side].ghost = __shfl(sd[side].ghost, src);
        }
        if (cl >= 0) ok = weno_group<M>(a, l, nmod, sc, ls, cl, cf, wout, xc) && ok;
      }
    }
  }
  if (!ok) atomicOr(a.err, (int)kErrState);
  if (a.advance) advance_step(a.step, par, n, blk == 0);
}

template <int M, int FLUX>
__global__ __launch_bounds__(kEulerBlock) void euler_stage_kernel(EulerArgs a) {
  euler_stage_body<M, FLUX, false>(a, LimiterArgs{}, nullptr, nullptr, blockIdx.x, a.par);
}

template <int M, int FLUX>
__global__ __launch_bounds__(kEulerBlock, M <= 4 ? 3 : 2) void euler_lim_kernel(EulerArgs a, LimiterArgs l) {
  __shared__ double lds[(kEulerBlock / 64) * lds_wave_doubles<M>()];
  __shared__ int rounds[kEulerBlock / 64];
  euler_stage_body<M, FLUX, true>(a, l, lds, rounds, blockIdx.x, a.par);
}

// Batched stage kernel: one workgroup per (instance, block) entry of the work
// list, for instances of one order, flux and limiter choice, all at step counter
// parity par; an instance whose step count has reached its target is skipped by
// all of its workgroups alike (its first one carries the count over to the
// other parity at the step's last stage).
template <int M, int FLUX, bool LIM>
__global__ __launch_bounds__(kEulerBlock, M <= 4 ? 3 : 2) void euler_batch_kernel(const EulerSet *__restrict__ sets,
                                                                  const int2 *__restrict__ tiles, int stage,
                                                                  int par) {
  const int2 tl = tiles[blockIdx.x];
  const EulerArgs &a = sets[tl.x].st[stage];
  const long long n = a.step[par];
  if (n >= a.target) {
    if (a.advance && tl.y == 0 && threadIdx.x == 0) a.step[par ^ 1] = n;
    return;
  }
  if constexpr (LIM) {
    __shared__ double lds[(kEulerBlock / 64) * lds_wave_doubles<M>()];
    __shared__ int rounds[kEulerBlock / 64];
    euler_stage_body<M, FLUX, true>(a, sets[tl.x].lim, lds, rounds, tl.y, par);
  } else {
    euler_stage_body<M, FLUX, false>(a, sets[tl.x].lim, nullptr, nullptr, tl.y, par);
  }
}

// caller layout [E][VM] <-> device layout (sidx)
__global__ void to_planes_kernel(const double *__restrict__ src, double *__restrict__ dst, int E, int VM) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)E * VM) return;
  const int e = (int)(idx / VM), c = (int)(idx % VM);
  dst[sidx(e, c, VM)] = src[idx];
}
__global__ void from_planes_kernel(const double *__restrict__ src, double *__restrict__ dst, int E, int VM) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)E * VM) return;
  const int e = (int)(idx / VM), c = (int)(idx % VM);
  dst[idx] = src[sidx(e, c, VM)];
}

// ---------------------------------------------------------------- launchers

template <int M>
static hipError_t stage_M(int flux, const EulerArgs &a, const LimiterArgs *lim, hipStream_t s) {
  const int blocks = euler_blocks(a.E, lim != nullptr);
  if (lim) {
    if (flux == 1) hipLaunchKernelGGL((euler_lim_kernel<M, 1>), dim3(blocks), dim3(kEulerBlock), 0, s, a, *lim);
    else hipLaunchKernelGGL((euler_lim_kernel<M, 0>), dim3(blocks), dim3(kEulerBlock), 0, s, a, *lim);
  } else {
    if (flux == 1) hipLaunchKernelGGL((euler_stage_kernel<M, 1>), dim3(blocks), dim3(kEulerBlock), 0, s, a);
    else hipLaunchKernelGGL((euler_stage_kernel<M, 0>), dim3(blocks), dim3(kEulerBlock), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_euler_stage(int M, int flux, const EulerArgs &a, const LimiterArgs *lim, hipStream_t s) {
  switch (M) {
    case 2: return stage_M<2>(flux, a, lim, s);
    case 3: return stage_M<3>(flux, a, lim, s);
    case 4: return stage_M<4>(flux, a, lim, s);
    case 5: return stage_M<5>(flux, a, lim, s);
  }
  return hipErrorInvalidValue;
}

template <int M, bool LIM>
static hipError_t batch_ML(int flux, const EulerSet *sets, const int2 *tiles, int ntiles, int stage, int par,
                           hipStream_t s) {
  if (flux == 1)
    hipLaunchKernelGGL((euler_batch_kernel<M, 1, LIM>), dim3(ntiles), dim3(kEulerBlock), 0, s, sets, tiles, stage, par);
  else
    hipLaunchKernelGGL((euler_batch_kernel<M, 0, LIM>), dim3(ntiles), dim3(kEulerBlock), 0, s, sets, tiles, stage, par);
  return hipGetLastError();
}

template <int M>
static hipError_t batch_M(int flux, bool lim, const EulerSet *sets, const int2 *tiles, int ntiles, int stage,
                          int par, hipStream_t s) {
  return lim ? batch_ML<M, true>(flux, sets, tiles, ntiles, stage, par, s)
             : batch_ML<M, false>(flux, sets, tiles, ntiles, stage, par, s);
}

hipError_t launch_euler_batch(int M, int flux, bool lim, const EulerSet *sets, const int2 *tiles, int ntiles,
                              int stage, int par, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  switch (M) {
    case 2: return batch_M<2>(flux, lim, sets, tiles, ntiles, stage, par, s);
    case 3: return batch_M<3>(flux, lim, sets, tiles, ntiles, stage, par, s);
    case 4: return batch_M<4>(flux, lim, sets, tiles, ntiles, stage, par, s);
    case 5: return batch_M<5>(flux, lim, sets, tiles, ntiles, stage, par, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_to_planes(const double *src, double *dst, int E, int VM, hipStream_t s) {
  const long long n = (long long)E * VM;
  hipLaunchKernelGGL(to_planes_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, E, VM);
  return hipGetLastError();
}

hipError_t launch_from_planes(const double *src, double *dst, int E, int VM, hipStream_t s) {
  const long long n = (long long)E * VM;
  hipLaunchKernelGGL(from_planes_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, E, VM);
  return hipGetLastError();
}

}  // namespace adg
