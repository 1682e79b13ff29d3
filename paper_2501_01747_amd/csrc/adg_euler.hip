// Fused SSP-RK3 stage kernel for the one-step reactive Euler model and the
// troubled-cell indicator + characteristic (AT-)WENO limiter (three passes:
// indicator over every element, WENO over the list of troubled elements,
// write-back of the limited values).
//
// Stage kernel (Sec. 3.1 Eq. (5), Sec. 3.2 Eq. (7)): one thread per element;
// each wavefront owns 62 consecutive elements and holds their two neighbours.
// Every lane loads its element's modal DoFs from the component planes
// (coalesced) and forms both face traces; one numerical flux per face is
// computed and passed to the neighbouring lane by a shuffle; at PE-interface
// faces the synchronous flux of this level is written to the history ring and
// replaced by the AT combination of past levels.  The volume integral, the
// source projection, the lift and the RK combination then run in registers and
// the output is stored once.  HBM traffic per stage: read w^(s) (+ w^n for
// stages 2 and 3), write w^(s+1).
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

// Numerical flux at a face from its two traces; at PE interface i the AT flux.
template <int FLUX>
__device__ __forceinline__ bool face_flux(const EulerArgs &a, long long n, int i, const double *wm,
                                          const double *wp, double *F) {
  bool ok = numflux1<FLUX>(a.ph, wm, wp, F);
  if (i >= 0) {
    double *rec = ring_rec(a.ring, n, a.stage, a.dl.nif, i) + a.ring.off_F;
#pragma unroll
    for (int v = 0; v < 5; ++v) rec[v] = F[v];
    const int k = eff_delay(a.dl, n, i);
    if (k > 0) {
      double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
      for (int j = 0; j < a.dl.q; ++j) {
        const double c = at_weight(a.dl.q, k, j);
        const double *h = ring_rec(a.ring, n - k - j, a.stage, a.dl.nif, i) + a.ring.off_F;
#pragma unroll
        for (int v = 0; v < 5; ++v) acc[v] += c * h[v];
      }
#pragma unroll
      for (int v = 0; v < 5; ++v) F[v] = acc[v];
    }
  }
  return ok;
}

// Wavefront-local stage kernel.  Lane l of a wavefront holds element
// base + l - 1 (base = 62 * wavefront index): lanes 1..62 own their element,
// lanes 0 and 63 hold the halo neighbours, loaded together with the owned
// elements.  Lane k computes the flux at the face between its element and lane
// k+1's; traces and fluxes move between lanes by cross-lane shuffles, so no
// LDS and no workgroup barrier is needed.
template <int M, int FLUX>
__device__ __forceinline__ void euler_stage_body(const EulerArgs &a, int blk, int nblk) {
  constexpr int V = 5, Q = M;
  const int lane = threadIdx.x & 63;
  const int base = ((blk * kEulerBlock + threadIdx.x) >> 6) * kWaveElems;
  const int E = a.E;
  const int xu = base + lane - 1;                       // element index before periodic wrap
  const bool live = base < E;
  const bool own = live && lane >= 1 && lane <= kWaveElems && xu < E;
  const bool ghost_l = !a.periodic && xu == -1;         // transmissive ends: ghost = interior trace
  const bool ghost_r = !a.periodic && xu == E;
  const bool loads = live && xu <= E && !ghost_l && !ghost_r;
  const bool face_lane = live && lane <= kWaveElems && xu + 1 <= E;  // face xu + 1 in [0, E]
  int x = xu % E;
  if (x < 0) x += E;
  const long long n = *a.step;
  bool ok = true;

  double u[V][M], wn[V][M];
  // the second operand of the RK combination of an owned element (w^n, or the 2N
  // register) is loaded together with the stage input, so both loads are in flight at
  // once (the last Shu-Osher stage overwrites w^n in place; only this lane reads it)
  const bool use_prev = own && (a.rk.two_n ? a.rk.ca != 0.0 : a.rk.ca != 0.0 || a.rk.cb != 1.0);
  if (use_prev) load_elem<M>(a.rk.two_n ? a.kbuf : a.w0, E, x, wn);
  if (loads) {
    load_elem<M>(a.ws, E, x, u);
  } else {
#pragma unroll
    for (int v = 0; v < V; ++v)
#pragma unroll
      for (int j = 0; j < M; ++j) u[v][j] = 0.0;
  }
  const int iface = face_lane ? a.face_if[xu + 1] : -1;

  double wl[V], wr[V];
  traces<M>(u, wl, wr);
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const double next_l = __shfl_down(wl[v], 1);
    const double prev_r = __shfl_up(wr[v], 1);
    if (ghost_l) wr[v] = next_l;
    if (ghost_r) wl[v] = prev_r;
  }
  // flux at the face to the right of this lane's element
  double F[V];
  {
    double wp[V];
#pragma unroll
    for (int v = 0; v < V; ++v) wp[v] = __shfl_down(wl[v], 1);
    const bool fok = face_flux<FLUX>(a, n, iface, wr, wp, F);
    if (face_lane) ok = fok && ok;
  }
  double Fl[V];
#pragma unroll
  for (int v = 0; v < V; ++v) Fl[v] = __shfl_up(F[v], 1);
  const int if_left = __shfl_up(iface, 1);

  if (own) {
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
    double *recR = (a.store_U && if_left >= 0)   // this element is right of interface if_left
                       ? ring_rec(a.ring, n, a.stage, a.dl.nif, if_left) + a.ring.off_U + V * M : nullptr;
    double *recL = (a.store_U && iface >= 0)     // left of interface iface
                       ? ring_rec(a.ring, n, a.stage, a.dl.nif, iface) + a.ring.off_U : nullptr;
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
          a.kbuf[gi] = kn;
          o = fma(a.rk.cb, kn, u[v][j]);
        } else {
          const double y = fma(a.dt, L, u[v][j]);
          o = use_prev ? fma(a.rk.ca, wn[v][j], a.rk.cb * y) : y;
        }
        a.wout[gi] = o;
        if (recR) recR[v * M + j] = o;
        if (recL) recL[v * M + j] = o;
      }
    }
  }
  if (!ok) atomicOr(a.err, (int)kErrState);
  if (a.advance) finish_step(a.step, a.done, nblk);
}

template <int M, int FLUX>
__global__ __launch_bounds__(kEulerBlock) void euler_stage_kernel(EulerArgs a) {
  euler_stage_body<M, FLUX>(a, blockIdx.x, gridDim.x);
}

__host__ __device__ inline int euler_blocks(int E) {
  const int waves = (E + kWaveElems - 1) / kWaveElems;
  return (waves + kEulerBlock / 64 - 1) / (kEulerBlock / 64);
}

// Batched stage kernel: one workgroup per (instance, block) entry of the work
// list, for instances of one order and flux; an instance whose step count has
// reached its target is skipped by all of its workgroups alike.
template <int M, int FLUX>
__global__ __launch_bounds__(kEulerBlock) void euler_batch_kernel(const EulerSet *__restrict__ sets,
                                                                  const int2 *__restrict__ tiles, int stage) {
  const int2 tl = tiles[blockIdx.x];
  const EulerArgs &a = sets[tl.x].st[stage];
  if (*a.step >= a.target) return;
  euler_stage_body<M, FLUX>(a, tl.y, euler_blocks(a.E));
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
  const double dp[5] = {g1 * 0.5 * u * u, -g1 * u, g1, -g1 * q, 0.0};
  const double du[5] = {-u / rho, 1.0 / rho, 0.0, 0.0, 0.0};
  const double a2 = a * a;
  const double YR = wb[3] / rho, YP = 1.0 - YR;
  const double l2[5] = {-YR, 0.0, 0.0, 1.0, 0.0};
  const double l3[5] = {-1.0, 0.0, 0.0, 1.0, 1.0};
  // the acoustic rows carry the sign of their wave speed u -+ a
  const double sa = c == 0 ? -1.0 : 1.0;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const double drho = k == 0 ? 1.0 : 0.0;
    const double ac = (dp[k] + sa * rho * a * du[k]) / (2.0 * a2);
    lr[k] = (c == 0 || c == 4) ? ac : c == 1 ? drho - dp[k] / a2 : c == 2 ? l2[k] : l3[k];
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

// Modal data of a neighbour: loaded from the unlimited stage output, the
// AT combination of Eq. (11) from the history ring, or the constant ghost.
template <int M>
__device__ void neighbour_modes(const LimiterArgs &a, long long n, int e, int side, const double (&u)[5][M],
                                double (&nb)[5][M]) {
  const int E = a.E;
  const bool ghost = !a.periodic && (side == 0 ? e == 0 : e == E - 1);
  if (ghost) {
#pragma unroll
    for (int v = 0; v < 5; ++v)
#pragma unroll
      for (int j = 0; j < M; ++j) nb[v][j] = j == 0 ? u[v][0] : 0.0;
    return;
  }
  const int face = side == 0 ? e : e + 1;
  const int i = a.face_if[face];
  const int k = i >= 0 ? eff_delay(a.dl, n, i) : 0;
  if (k > 0) {
#pragma unroll
    for (int v = 0; v < 5; ++v)
#pragma unroll
      for (int j = 0; j < M; ++j) nb[v][j] = 0.0;
    // side 0: the neighbour is the element left of interface i (record slot 0)
    const int off = a.ring.off_U + (side == 0 ? 0 : 5 * M);
    for (int jj = 0; jj < a.dl.q; ++jj) {
      const double c = at_weight(a.dl.q, k, jj);
      const double *h = ring_rec(a.ring, n - k - jj, a.stage, a.dl.nif, i) + off;
#pragma unroll
      for (int v = 0; v < 5; ++v)
#pragma unroll
        for (int j = 0; j < M; ++j) nb[v][j] += c * h[v * M + j];
    }
    return;
  }
  const int en = side == 0 ? (e == 0 ? E - 1 : e - 1) : (e == E - 1 ? 0 : e + 1);
  load_elem<M>(a.w, E, en, nb);
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

// Neighbour data of element e for the limiter: its two neighbours' modes (Eq. (11)
// data across delayed PE faces, the constant ghost at transmissive ends).
template <int M>
__device__ __forceinline__ void limiter_stencil(const LimiterArgs &a, long long n, int e, double (&u)[5][M],
                                                double (&nbL)[5][M], double (&nbR)[5][M]) {
  load_elem<M>(a.w, a.E, e, u);
  neighbour_modes<M>(a, n, e, 0, u, nbL);
  neighbour_modes<M>(a, n, e, 1, u, nbR);
}

// Troubled-cell indicator of element e (KXRCF or TVB minmod).
template <int M>
__device__ __forceinline__ bool troubled(const LimiterArgs &a, int e, const double (&u)[5][M],
                                         const double (&nbL)[5][M], const double (&nbR)[5][M]) {
  const bool ghostL = !a.periodic && e == 0, ghostR = !a.periodic && e == a.E - 1;
  bool flag = false;
  if (a.indicator == 1) {
    // TVB minmod: the face deviations from the mean against the mean differences, every
    // variable; differences within 1e-10 of the largest |mean| of any variable in the
    // stencil count as equal (round-off in a constant state is not a slope)
    double scale = 0.0;
#pragma unroll
    for (int v = 0; v < 5; ++v) scale = fmax(scale, fmax(fabs(u[v][0]), fmax(fabs(nbL[v][0]), fabs(nbR[v][0]))));
    const double tol = 1e-10 * scale;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const double m = u[v][0], mL = nbL[v][0], mR = nbR[v][0];
      const double dp = trace_at<M>(u[v], 1) - m, dm = m - trace_at<M>(u[v], 0);
      const double Dp = mR - m, Dm = m - mL;
      const double mp = fabs(dp) <= a.tvb_mh2 ? dp : minmod3(dp, Dp, Dm);
      const double mm = fabs(dm) <= a.tvb_mh2 ? dm : minmod3(dm, Dp, Dm);
      if (fabs(mp - dp) > tol || fabs(mm - dm) > tol) flag = true;
    }
  } else {
  // KXRCF: jumps at inflow faces against h^((N_p+1)/2) max_q |w(xi_q)|, on rho and rho E.
  const double uL_e = trace_at<M>(u[1], 0) / trace_at<M>(u[0], 0);
  const double uR_e = trace_at<M>(u[1], 1) / trace_at<M>(u[0], 1);
  const double uL_n = ghostL ? uL_e : trace_at<M>(nbL[1], 1) / trace_at<M>(nbL[0], 1);
  const double uR_n = ghostR ? uR_e : trace_at<M>(nbR[1], 0) / trace_at<M>(nbR[0], 0);
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int v = t == 0 ? 0 : 2;
    double jump = 0.0;
    if (0.5 * (uL_e + uL_n) > 0.0 && !ghostL) jump += trace_at<M>(u[v], 0) - trace_at<M>(nbL[v], 1);
    if (0.5 * (uR_e + uR_n) < 0.0 && !ghostR) jump += trace_at<M>(u[v], 1) - trace_at<M>(nbR[v], 0);
    double norm = 0.0;
#pragma unroll
    for (int q = 0; q < M; ++q) {
      double val = 0.0;
#pragma unroll
      for (int j = 0; j < M; ++j) val += u[v][j] * a.tb.B[q][j];
      norm = fmax(norm, fabs(val));
    }
    if (fabs(jump) / (a.kx_h * norm) > 1.0) flag = true;
  }
  }
  return flag;
}

// Pass 1 of the limiter, every element: the indicator; troubled elements are
// appended to the stage's list (their order does not matter: each is limited on
// its own in pass 2).
template <int M>
__device__ __forceinline__ void indicator_body(const LimiterArgs &a, int blk) {
  const int e = blk * kLimBlock + threadIdx.x;
  if (e >= a.E) return;
  const long long n = *a.step;
  double u[5][M], nbL[5][M], nbR[5][M];
  limiter_stencil<M>(a, n, e, u, nbL, nbR);
  const bool flag = troubled<M>(a, e, u, nbL, nbR);
  a.flags[e] = flag ? 1 : 0;
  if (flag) {
    atomicAdd(a.flag_count, 1ull);
    a.tlist[atomicAdd(a.tcount + a.stage, 1u)] = e;
  }
}

// The simple WENO reconstruction of Eq. (9)-(10) of one characteristic field (L row
// lr): the limited modes vl of that field in the cell.
template <int M>
__device__ __forceinline__ void weno_field(const LimiterArgs &a, const double (&lr)[5], const double (&u)[5][M],
                                           const double (&nbL)[5][M], const double (&nbR)[5][M], double (&vl)[M]) {
  double vc[M], vL[M], vR[M];
#pragma unroll
  for (int j = 0; j < M; ++j) {
    double x0 = 0.0, xl = 0.0, xr = 0.0;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      x0 += lr[v] * u[v][j];
      xl += lr[v] * nbL[v][j];
      xr += lr[v] * nbR[v][j];
    }
    vc[j] = x0; vL[j] = xl; vR[j] = xr;
  }
  // re-expand the neighbours in the cell's coordinate and reset their mean
  double tL[M], tR[M];
#pragma unroll
  for (int k2 = 0; k2 < M; ++k2) {
    double sl = 0.0, sr = 0.0;
#pragma unroll
    for (int j = 0; j < M; ++j) {
      sl += a.Tl[k2][j] * vL[j];
      sr += a.Tr[k2][j] * vR[j];
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
      beta[0] += tL[p] * a.Bm[p][r] * tL[r];
      beta[1] += vc[p] * a.Bm[p][r] * vc[r];
      beta[2] += tR[p] * a.Bm[p][r] * tR[r];
    }
  double wbar[3], sum = 0.0;
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const double d = a.eps + beta[s];
    wbar[s] = a.gam[s] / (d * d);
    sum += wbar[s];
  }
  const double om0 = wbar[0] / sum, om1 = wbar[1] / sum, om2 = wbar[2] / sum;
#pragma unroll
  for (int j = 0; j < M; ++j) vl[j] = om0 * tL[j] + om1 * vc[j] + om2 * tR[j];
}

// Pass 2, the listed elements only (grid-stride over the list), characteristic WENO
// into the side buffer.  A group of kWenoGroup lanes per troubled element: lane c < 5
// limits characteristic field c, and w_lim = sum_c R[:, c] v_c^lim is summed across
// the group in a fixed butterfly order (lanes 5..7 add zeros).
template <int M>
__device__ __forceinline__ void weno_body(const LimiterArgs &a, int blk, int nblk) {
  constexpr int G = kWenoGroup, per = kWenoBlock / G;
  const unsigned cnt = a.tcount[a.stage];
  if ((unsigned)(blk * per) >= cnt) return;
  const long long n = *a.step;
  const int c = threadIdx.x % G;
  const int cf = c < 5 ? c : 4;
  // idx is uniform within a group, so the shuffles below see all G lanes
  for (unsigned idx = blk * per + threadIdx.x / G; idx < cnt; idx += nblk * per) {
    const int e = a.tlist[idx];
    double u[5][M], nbL[5][M], nbR[5][M];
    limiter_stencil<M>(a, n, e, u, nbL, nbR);
    double wb[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) wb[v] = u[v][0];
    double lr[5], rc[5];
    if (!char_row_col(a.ph, wb, cf, lr, rc) && c == 0) atomicOr(a.err, (int)kErrState);
    double vl[M];
    weno_field<M>(a, lr, u, nbL, nbR, vl);
#pragma unroll
    for (int v = 0; v < 5; ++v)
#pragma unroll
      for (int j = 0; j < M; ++j) {
        double part = c < 5 ? rc[v] * vl[j] : 0.0;
#pragma unroll
        for (int m = 1; m < G; m <<= 1) part += __shfl_xor(part, m, G);
        if (c == v) a.wlim[sidx(e, v * M + j, 5 * M)] = part;
      }
  }
}

template <int M>
__global__ __launch_bounds__(kLimBlock) void limiter_kernel(LimiterArgs a) {
  indicator_body<M>(a, blockIdx.x);
}

template <int M>
__global__ __launch_bounds__(kLimBlock) void limiter_batch_kernel(const EulerSet *__restrict__ sets,
                                                                  const int2 *__restrict__ tiles, int stage) {
  const int2 tl = tiles[blockIdx.x];
  const LimiterArgs &a = sets[tl.x].lim[stage];
  if (*a.step >= a.target) return;
  indicator_body<M>(a, tl.y);
}

template <int M>
__global__ __launch_bounds__(kWenoBlock) void weno_kernel(LimiterArgs a) {
  weno_body<M>(a, blockIdx.x, gridDim.x);
}

template <int M>
__global__ __launch_bounds__(kWenoBlock) void weno_batch_kernel(const EulerSet *__restrict__ sets,
                                                                const int2 *__restrict__ tiles, int stage) {
  const int2 tl = tiles[blockIdx.x];
  const LimiterArgs &a = sets[tl.x].lim[stage];
  if (*a.step >= a.target) return;
  weno_body<M>(a, tl.y, weno_blocks(a.E));
}

// Pass 3, after every stencil has read the unlimited data: the limited values of
// the listed elements replace the unlimited ones.  The next stage's list starts
// empty; the last kernel of a step advances the step counter.
template <int M>
__device__ __forceinline__ void scatter_body(const LimiterArgs &a, int blk, int nblk) {
  const unsigned cnt = a.tcount[a.stage];
  for (unsigned idx = blk * kScatterBlock + threadIdx.x; idx < cnt; idx += nblk * kScatterBlock) {
    const int e = a.tlist[idx];
#pragma unroll
    for (int v = 0; v < 5; ++v)
#pragma unroll
      for (int j = 0; j < M; ++j) {
        const size_t gi = sidx(e, v * M + j, 5 * M);
        a.w[gi] = a.wlim[gi];
      }
  }
  if (blk == 0 && threadIdx.x == 0) a.tcount[(a.stage + 1) % a.nstages] = 0u;
  if (a.advance) finish_step(a.step, a.done, nblk);
}

template <int M>
__global__ __launch_bounds__(kScatterBlock) void limiter_scatter_kernel(LimiterArgs a) {
  scatter_body<M>(a, blockIdx.x, gridDim.x);
}

template <int M>
__global__ __launch_bounds__(kScatterBlock) void scatter_batch_kernel(const EulerSet *__restrict__ sets,
                                                                      const int2 *__restrict__ tiles, int stage) {
  const int2 tl = tiles[blockIdx.x];
  const LimiterArgs &a = sets[tl.x].lim[stage];
  if (*a.step >= a.target) return;
  scatter_body<M>(a, tl.y, scatter_blocks(a.E));
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
static hipError_t stage_M(int flux, const EulerArgs &a, hipStream_t s) {
  const int blocks = euler_blocks(a.E);
  if (flux == 1) hipLaunchKernelGGL((euler_stage_kernel<M, 1>), dim3(blocks), dim3(kEulerBlock), 0, s, a);
  else hipLaunchKernelGGL((euler_stage_kernel<M, 0>), dim3(blocks), dim3(kEulerBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_euler_stage(int M, int flux, const EulerArgs &a, hipStream_t s) {
  switch (M) {
    case 2: return stage_M<2>(flux, a, s);
    case 3: return stage_M<3>(flux, a, s);
    case 4: return stage_M<4>(flux, a, s);
    case 5: return stage_M<5>(flux, a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_limiter(int M, const LimiterArgs &a, hipStream_t s) {
  const int blocks = (a.E + kLimBlock - 1) / kLimBlock;
  switch (M) {
    case 2: hipLaunchKernelGGL(limiter_kernel<2>, dim3(blocks), dim3(kLimBlock), 0, s, a); break;
    case 3: hipLaunchKernelGGL(limiter_kernel<3>, dim3(blocks), dim3(kLimBlock), 0, s, a); break;
    case 4: hipLaunchKernelGGL(limiter_kernel<4>, dim3(blocks), dim3(kLimBlock), 0, s, a); break;
    case 5: hipLaunchKernelGGL(limiter_kernel<5>, dim3(blocks), dim3(kLimBlock), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_weno(int M, const LimiterArgs &a, hipStream_t s) {
  const int blocks = weno_blocks(a.E);
  switch (M) {
    case 2: hipLaunchKernelGGL(weno_kernel<2>, dim3(blocks), dim3(kWenoBlock), 0, s, a); break;
    case 3: hipLaunchKernelGGL(weno_kernel<3>, dim3(blocks), dim3(kWenoBlock), 0, s, a); break;
    case 4: hipLaunchKernelGGL(weno_kernel<4>, dim3(blocks), dim3(kWenoBlock), 0, s, a); break;
    case 5: hipLaunchKernelGGL(weno_kernel<5>, dim3(blocks), dim3(kWenoBlock), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_limiter_scatter(int M, const LimiterArgs &a, hipStream_t s) {
  const int blocks = scatter_blocks(a.E);
  switch (M) {
    case 2: hipLaunchKernelGGL(limiter_scatter_kernel<2>, dim3(blocks), dim3(kScatterBlock), 0, s, a); break;
    case 3: hipLaunchKernelGGL(limiter_scatter_kernel<3>, dim3(blocks), dim3(kScatterBlock), 0, s, a); break;
    case 4: hipLaunchKernelGGL(limiter_scatter_kernel<4>, dim3(blocks), dim3(kScatterBlock), 0, s, a); break;
    case 5: hipLaunchKernelGGL(limiter_scatter_kernel<5>, dim3(blocks), dim3(kScatterBlock), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int euler_batch_blocks(int kind, int E) {
  if (kind == 0) return euler_blocks(E);
  if (kind == 1) return (E + kLimBlock - 1) / kLimBlock;
  if (kind == 2) return weno_blocks(E);
  return scatter_blocks(E);
}

template <int M>
static hipError_t batch_M(int kind, int flux, const EulerSet *sets, const int2 *tiles, int ntiles, int stage,
                          hipStream_t s) {
  if (kind == 0) {
    if (flux == 1)
      hipLaunchKernelGGL((euler_batch_kernel<M, 1>), dim3(ntiles), dim3(kEulerBlock), 0, s, sets, tiles, stage);
    else
      hipLaunchKernelGGL((euler_batch_kernel<M, 0>), dim3(ntiles), dim3(kEulerBlock), 0, s, sets, tiles, stage);
  } else if (kind == 1) {
    hipLaunchKernelGGL(limiter_batch_kernel<M>, dim3(ntiles), dim3(kLimBlock), 0, s, sets, tiles, stage);
  } else if (kind == 2) {
    hipLaunchKernelGGL(weno_batch_kernel<M>, dim3(ntiles), dim3(kWenoBlock), 0, s, sets, tiles, stage);
  } else {
    hipLaunchKernelGGL(scatter_batch_kernel<M>, dim3(ntiles), dim3(kScatterBlock), 0, s, sets, tiles, stage);
  }
  return hipGetLastError();
}

hipError_t launch_euler_batch(int kind, int M, int flux, const EulerSet *sets, const int2 *tiles, int ntiles,
                              int stage, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  switch (M) {
    case 2: return batch_M<2>(kind, flux, sets, tiles, ntiles, stage, s);
    case 3: return batch_M<3>(kind, flux, sets, tiles, ntiles, stage, s);
    case 4: return batch_M<4>(kind, flux, sets, tiles, ntiles, stage, s);
    case 5: return batch_M<5>(kind, flux, sets, tiles, ntiles, stage, s);
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
