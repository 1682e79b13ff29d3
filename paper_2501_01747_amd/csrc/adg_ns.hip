// Fused SSP-RK3 stage kernel for the detailed-chemistry Navier-Stokes model
// (Sec. 2 Eq. (1)-(3), Sec. 3.1 LDG form of Eq. (5), Sec. 3.2 AT fluxes).
//
// One workgroup per tile of kTile elements, periodic domain.  The tile and a
// halo of two elements on each side are staged in LDS; every later phase reads
// LDS only:
//   1. face traces of w for the tile and halo;
//   2. central traces w* at the faces; at PE interfaces the synchronous w* of
//      this level goes to the history ring and the element-side w* becomes the
//      AT combination of past levels (Eq. (7) applied to w*);
//   3. LDG gradients q (modal) of the tile and one halo element per side;
//   4. one lane per point (quadrature nodes of the tile, both traces of every
//      tile face): temperature Newton, primitives, convective and diffusive
//      fluxes, and at the nodes the mass-action chemistry (FP64 throughout);
//   5. Rusanov total flux per face; at PE interfaces the synchronous flux goes
//      to the ring and the AT combination replaces it;
//   6. volume and source projection, lift and SSP-RK3 combination; the output
//      is stored once.
#include "adg_device.hpp"
#include "adg_ns.hpp"

#include <cmath>
#include <cstring>

namespace adg {

constexpr int kTile = 8;
constexpr int kThreads = 256;

template <int NS>
struct Thermo {
  double T, cp, cv, p, a;
  double hRT[NS];    // h_i / (R_i T)
  double eR[NS];     // e_i / R_i = T (h/(R T) - 1)
};

// Temperature from the internal energy by Newton's method from the fixed start
// T_guess, |dT| <= 1e-12 T; then the thermodynamic state at that T.  The
// mixture energy sum_i Y_i e_i(T) is linear in the species, so its polynomial
// coefficients are formed once per point and the iteration runs on one
// quintic: e(T)/1 = T (c0 + T (c1 + T (c2 + T (c3 + T c4)))) + c5.
template <int NS>
__device__ __forceinline__ bool ns_thermo(const NsMech *__restrict__ mk, const double *Y, double rho, double estar,
                                          Thermo<NS> &th) {
  double c0 = 0.0, c1 = 0.0, c2 = 0.0, c3 = 0.0, c4 = 0.0, c5 = 0.0, Rmix = 0.0;
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    const double yr = Y[i] * mk->Ri[i];
    c0 += yr * (mk->a[i][0] - 1.0);
    c1 += yr * mk->h2[i][0];
    c2 += yr * mk->h2[i][1];
    c3 += yr * mk->h2[i][2];
    c4 += yr * mk->h2[i][3];
    c5 += yr * mk->a[i][5];
    Rmix += yr;
  }
  // de/dT = c0 + 2 c1 T + 3 c2 T^2 + 4 c3 T^3 + 5 c4 T^4 = cv
  const double d1 = 2.0 * c1, d2 = 3.0 * c2, d3 = 4.0 * c3, d4 = 5.0 * c4;
  double T = mk->T_guess;
  bool conv = false;
  for (int it = 0; it < 50; ++it) {
    const double e = T * (c0 + T * (c1 + T * (c2 + T * (c3 + T * c4)))) + c5;
    const double cv = c0 + T * (d1 + T * (d2 + T * (d3 + T * d4)));
    const double dT = (e - estar) / cv;
    T -= dT;
    if (!(T > 0.0) || !isfinite(T)) break;
    if (fabs(dT) <= 1e-12 * T) { conv = true; break; }
  }
  th.T = T;
  const double invT = 1.0 / T;
  const double cv = c0 + T * (d1 + T * (d2 + T * (d3 + T * d4)));
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    const double *a = mk->a[i];
    const double *h2 = mk->h2[i];
    const double hT = T * (a[0] + T * (h2[0] + T * (h2[1] + T * (h2[2] + T * h2[3])))) + a[5];
    th.hRT[i] = hT * invT;
    th.eR[i] = hT - T;
  }
  th.cv = cv;
  th.cp = cv + Rmix;
  th.p = rho * Rmix * T;
  th.a = sqrt(th.cp / cv * th.p / rho);
  return conv && th.p > 0.0 && isfinite(th.p) && rho > 0.0;
}

// f^d of Eq. (2)-(3) with unit Lewis number: J_i = -rho D dY_i/dx, rho D = mu/Pr.
template <int NS>
__device__ __forceinline__ void ns_diffusive(const NsMech *__restrict__ mk, const double *w, const double *Y, double u,
                                             double rho_inv, const Thermo<NS> &th, double mu, const double *dw,
                                             double *fd) {
  const double kappa = mu * th.cp * mk->inv_prandtl;
  const double rhoD = mu * mk->inv_prandtl;
  const double u_x = (dw[1] - u * dw[0]) * rho_inv;
  const double E = w[2] * rho_inv;
  const double e_x = (dw[2] - E * dw[0]) * rho_inv - u * u_x;
  double sum_eY = 0.0, sum_hJ = 0.0;
  double Jm[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    const double Yx = (dw[3 + i] - Y[i] * dw[0]) * rho_inv;
    sum_eY += mk->Ri[i] * th.eR[i] * Yx;
    const double J = -rhoD * Yx;
    Jm[i] = J;
    sum_hJ += mk->Ri[i] * th.T * th.hRT[i] * J;
  }
  const double T_x = (e_x - sum_eY) / th.cv;
  const double tau = (4.0 / 3.0) * mu * u_x;
  const double qh = -kappa * T_x + sum_hJ;
  fd[0] = 0.0;
  fd[1] = tau;
  fd[2] = tau * u - qh;
#pragma unroll
  for (int i = 0; i < NS; ++i) fd[3 + i] = -Jm[i];
}

// Mass-action source W_i omega_i of the reversible mechanism.
template <int NS>
__device__ __forceinline__ void ns_source(const NsMech *__restrict__ mk, const double *rhoY, double T, double *src) {
  const double lnT = log(T);
  const double invT = 1.0 / T;
  double gRT[NS], conc[NS], wdot[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    const double *a = mk->a[i];
    const double *h2 = mk->h2[i];
    const double *s2 = mk->s2[i];
    const double hRT = a[0] + T * (h2[0] + T * (h2[1] + T * (h2[2] + T * h2[3]))) + a[5] * invT;
    const double sR = a[0] * lnT + T * (a[1] + T * (s2[0] + T * (s2[1] + T * s2[2]))) + a[6];
    gRT[i] = hRT - sR;
    conc[i] = rhoY[i] * mk->invW[i];
    wdot[i] = 0.0;
  }
  const double ln_pRT = mk->ln_p_over_Ru - lnT;   // ln(p_ref / (Ru T))
  for (int r = 0; r < mk->nr; ++r) {
    const double lnkf = mk->lnA[r] + mk->b[r] * lnT - mk->EaR[r] * invT;
    double dG = 0.0;
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      const int nu = mk->nur[r][i] - mk->nuf[r][i];
      if (nu != 0) dG += (double)nu * gRT[i];
    }
    const double lnKc = -dG + (double)mk->dnu[r] * ln_pRT;
    double fwd = exp(lnkf), rev = exp(lnkf - lnKc);
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      const int f = mk->nuf[r][i], b = mk->nur[r][i];
      if (f >= 1) fwd *= conc[i];
      if (f >= 2) fwd *= conc[i];
      if (b >= 1) rev *= conc[i];
      if (b >= 2) rev *= conc[i];
    }
    const double q = fwd - rev;
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      const int nu = mk->nur[r][i] - mk->nuf[r][i];
      if (nu != 0) wdot[i] += (double)nu * q;
    }
  }
#pragma unroll
  for (int i = 0; i < NS; ++i) src[i] = mk->W[i] * wdot[i];
}

// Everything but the chemistry evaluated at one point: g = f^c - f^d (and
// g_sync with the synchronous gradient when dw_sync is given), the spectral
// radius |u| + a and the temperature.
template <int NS>
__device__ __forceinline__ bool ns_point(const NsMech *__restrict__ mk, int viscous, const double (&w)[3 + NS],
                                         const double (&dw)[3 + NS], bool sync, const double (&dw_sync)[3 + NS],
                                         double (&g)[3 + NS], double (&g_sync)[3 + NS], double &lam, double &T) {
  constexpr int V = 3 + NS;
  const double rho = w[0];
  const double rho_inv = 1.0 / rho;
  const double u = w[1] * rho_inv;
  double Y[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) Y[i] = w[3 + i] * rho_inv;
  const double estar = w[2] * rho_inv - 0.5 * u * u;
  Thermo<NS> th;
  const bool ok = ns_thermo<NS>(mk, Y, rho, estar, th);
  lam = fabs(u) + th.a;
  g[0] = w[1];
  g[1] = w[1] * u + th.p;
  g[2] = u * (w[2] + th.p);
#pragma unroll
  for (int i = 0; i < NS; ++i) g[3 + i] = w[3 + i] * u;
#pragma unroll
  for (int v = 0; v < V; ++v) g_sync[v] = g[v];
  if (viscous) {
    const double mu = mk->mu_ref * exp(mk->mu_exp * log(th.T * mk->inv_T_ref));
    double fd[V];
    ns_diffusive<NS>(mk, w, Y, u, rho_inv, th, mu, dw, fd);
#pragma unroll
    for (int v = 0; v < V; ++v) g[v] -= fd[v];
    if (sync) {
      ns_diffusive<NS>(mk, w, Y, u, rho_inv, th, mu, dw_sync, fd);
#pragma unroll
      for (int v = 0; v < V; ++v) g_sync[v] -= fd[v];
    }
  }
  T = th.T;
  return ok;
}

template <int M, int NS>
__global__ __launch_bounds__(kThreads) void ns_stage_kernel(NsArgs a) {
  constexpr int V = 3 + NS, Q = M, TE = kTile;
  constexpr int NH = TE + 4;   // tile + 2 halo elements per side; local l <-> element e0 - 2 + l
  constexpr int NF = TE + 3;   // faces e0-1 .. e0+TE+1; local fl <-> face e0 - 1 + fl
  constexpr int NQ = TE + 2;   // gradients of elements e0-1 .. e0+TE; local lq <-> element e0 - 1 + lq
  constexpr int NN = TE * Q;   // quadrature nodes of the tile; node p <-> element p / Q, node p % Q
  constexpr int NT = 2 * (TE + 1);  // face traces; trace pp <-> face e0 + pp/2, side pp%2
  constexpr int NR = kNsMaxReactions;
  static_assert(NN <= 64 && NT <= 64, "node and trace lanes each fit one wavefront");
  __shared__ double sW[V * M][NH];
  __shared__ double sTm[V][NH], sTp[V][NH];
  __shared__ double sWc[V][NF], sWa[V][NF];
  __shared__ double sQ[V * M][NQ];
  __shared__ double sG[V][NN];
  __shared__ double sS[NS][NN];
  __shared__ double sT[NN];
  __shared__ double sConc[NS][NN], sGRT[NS][NN];
  __shared__ double sRate[NR][NN];
  __shared__ double sGf[2][V][TE + 1], sGs[2][V][TE + 1];
  __shared__ double sLam[2][TE + 1];
  __shared__ double sF[V][TE + 1], sFat[V][TE + 1];
  __shared__ int sI[NF], sK[NF];
  __shared__ double sB[Q][M], sWG[Q][M], sWB[Q][M], sD[M][M];   // tables, indexed at run time

  const int t = threadIdx.x;
  const int E = a.E;
  const int e0 = blockIdx.x * TE;
  const int nloc = min(TE, E - e0);
  const long long n = *a.step;
  __shared__ NsMech smech;
  const NsMech *__restrict__ mk = &smech;
  const int q_at = a.dl.q;
  bool ok = true;

  // 0. mechanism, state of the tile and its halo, tables, PE-interface data of the faces
  {
    const unsigned long long *src = reinterpret_cast<const unsigned long long *>(a.mech);
    unsigned long long *dst = reinterpret_cast<unsigned long long *>(&smech);
    constexpr int nwords = (int)(sizeof(NsMech) / 8);
    for (int idx = t; idx < nwords; idx += kThreads) dst[idx] = src[idx];
  }
#pragma unroll 3
  for (int idx = t; idx < V * M * NH; idx += kThreads) {
    const int c = idx / NH, l = idx % NH;
    int e = (e0 - 2 + l) % E;
    if (e < 0) e += E;
    sW[c][l] = a.ws[sidx(e, c, V * M)];
  }
  for (int idx = t; idx < Q * M; idx += kThreads) {
    const int qn = idx / M, j = idx % M;
    sB[qn][j] = a.tb.B[qn][j];
    sWG[qn][j] = a.tb.WG[qn][j];
    sWB[qn][j] = a.tb.WB[qn][j];
    if (qn < M) sD[qn][j] = a.tb.Dm[qn][j];
  }
  for (int fl = t; fl < NF; fl += kThreads) {
    int f = (e0 - 1 + fl) % E;
    if (f < 0) f += E;
    const int i = a.face_if[f];
    sI[fl] = i;
    sK[fl] = i >= 0 ? eff_delay(a.dl, n, i) : 0;
  }
  __syncthreads();
  const int nr = mk->nr;

  // 1. traces of w; meanwhile the AT combinations of past levels (Eq. (7)) of the central
  //    traces and of the fluxes at delayed PE interfaces are gathered from the ring
  for (int idx = t; idx < V * NH; idx += kThreads) {
    const int v = idx / NH, l = idx % NH;
    double sm = 0.0, sp = 0.0;
#pragma unroll
    for (int j = 0; j < M; ++j) {
      const double c = sW[v * M + j][l];
      sp += c;
      sm += (j & 1) ? -c : c;
    }
    sTm[v][l] = sm;
    sTp[v][l] = sp;
  }
  for (int idx = t; idx < V * NF; idx += kThreads) {
    const int v = idx / NF, fl = idx % NF;
    const int i = sI[fl], k = sK[fl];
    if (i < 0 || k == 0) continue;
    double acw = 0.0, acf = 0.0;
    for (int j = 0; j < q_at; ++j) {
      const double c = at_weight(q_at, k, j);
      const double *rec = ring_rec(a.ring, n - k - j, a.stage, a.dl.nif, i);
      acw += c * rec[a.ring.off_Wc + v];
      acf += c * rec[a.ring.off_F + v];
    }
    sWa[v][fl] = acw;
    if (fl >= 1 && fl <= TE + 1) sFat[v][fl - 1] = acf;
  }
  __syncthreads();

  // 2. central traces; face fl sits between local elements fl (left) and fl + 1 (right).
  //    The synchronous value of a PE interface is published for this level.
  for (int idx = t; idx < V * NF; idx += kThreads) {
    const int v = idx / NF, fl = idx % NF;
    const double wc = 0.5 * (sTp[v][fl] + sTm[v][fl + 1]);
    const int i = sI[fl];
    if (i >= 0 && fl >= 1 && fl <= nloc)   // faces e0 .. e0+nloc-1 are owned by this tile
      ring_rec(a.ring, n, a.stage, a.dl.nif, i)[a.ring.off_Wc + v] = wc;
    sWc[v][fl] = wc;
    if (i < 0 || sK[fl] == 0) sWa[v][fl] = wc;
  }
  __syncthreads();

  // 3. LDG gradient q_j = (2j+1)/dx [w*_R - (-1)^j w*_L - sum_k D_jk w_k] of the element
  //    with gradient slot lq (left face lq, right face lq + 1)
  for (int idx = t; idx < V * M * NQ; idx += kThreads) {
    const int c = idx / NQ, lq = idx % NQ;
    const int v = c / M, j = c % M;
    double vol = 0.0;
#pragma unroll
    for (int k = 0; k < M; ++k) vol += sD[j][k] * sW[v * M + k][lq + 1];
    const double wl = (j & 1) ? -sWa[v][lq] : sWa[v][lq];
    sQ[c][lq] = (2 * j + 1) * a.inv_dx * (sWa[v][lq + 1] - wl - vol);
  }
  __syncthreads();

  // 4a. point evaluations: wavefront 0 takes the quadrature nodes, wavefront 1 the face traces
  if (t < NN) {
    const int el = t / Q, qn = t % Q;
    double w[V], dw[V], g[V], gs[V], lam, T;
#pragma unroll
    for (int v = 0; v < V; ++v) {
      double x = 0.0, d = 0.0;
#pragma unroll
      for (int j = 0; j < M; ++j) {
        x += sB[qn][j] * sW[v * M + j][el + 2];
        d += sB[qn][j] * sQ[v * M + j][el + 1];
      }
      w[v] = x;
      dw[v] = d;
    }
    ok = ns_point<NS>(mk, a.viscous, w, dw, false, dw, g, gs, lam, T) && ok;
#pragma unroll
    for (int v = 0; v < V; ++v) sG[v][t] = g[v];
    sT[t] = T;
  } else if (t >= 64 && t < 64 + NT) {
    const int pp = t - 64;
    const int ff = pp >> 1, side = pp & 1;  // face e0 + ff; side 0 = element left of it (at xi = +1)
    const int l = ff + 1 + side;            // local element
    const int lq = ff + side;               // its gradient slot; faces lq (left), lq + 1 (right)
    const double sgn = side ? -1.0 : 1.0;   // P_j(+-1) = (+-1)^j
    double w[V], dw[V], g[V], gs[V], dws[V], lam, T;
#pragma unroll
    for (int v = 0; v < V; ++v) {
      w[v] = side ? sTm[v][l] : sTp[v][l];
      double d = 0.0, pj = 1.0;
#pragma unroll
      for (int j = 0; j < M; ++j) {
        d += pj * sQ[v * M + j][lq];
        pj *= sgn;
      }
      dw[v] = d;
      dws[v] = d;
    }
    const bool pe = sI[ff + 1] >= 0;
    if (pe) {
      // synchronous gradient trace: undo the AT central traces of this element's faces
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const double dl = sWc[v][lq] - sWa[v][lq], dr = sWc[v][lq + 1] - sWa[v][lq + 1];
        double corr = 0.0, pj = 1.0;
#pragma unroll
        for (int j = 0; j < M; ++j) {
          corr += pj * (2 * j + 1) * a.inv_dx * (dr - ((j & 1) ? -dl : dl));
          pj *= sgn;
        }
        dws[v] = dw[v] + corr;
      }
    }
    ok = ns_point<NS>(mk, a.viscous, w, dw, pe, dws, g, gs, lam, T) && ok;
#pragma unroll
    for (int v = 0; v < V; ++v) {
      sGf[side][v][ff] = g[v];
      if (pe) sGs[side][v][ff] = gs[v];
    }
    sLam[side][ff] = lam;
  }
  __syncthreads();

  // 4b. chemistry (Sec. 2: W_i omega_i), one lane per (node, species), then one lane per
  //     (node, reaction), then one lane per (node, species) again
  for (int idx = t; idx < NS * NN; idx += kThreads) {
    const int i = idx / NN, p = idx % NN;
    const int el = p / Q, qn = p % Q;
    double x = 0.0;
#pragma unroll
    for (int j = 0; j < M; ++j) x += sB[qn][j] * sW[(3 + i) * M + j][el + 2];
    const double T = sT[p];
    const double lnT = log(T);
    const double *c = mk->a[i];
    const double *h2 = mk->h2[i];
    const double *s2 = mk->s2[i];
    const double hRT = c[0] + T * (h2[0] + T * (h2[1] + T * (h2[2] + T * h2[3]))) + c[5] / T;
    const double sR = c[0] * lnT + T * (c[1] + T * (s2[0] + T * (s2[1] + T * s2[2]))) + c[6];
    sGRT[i][p] = hRT - sR;
    sConc[i][p] = x * mk->invW[i];
  }
  __syncthreads();
  for (int idx = t; idx < nr * NN; idx += kThreads) {
    const int r = idx / NN, p = idx % NN;
    const double T = sT[p];
    const double lnT = log(T);
    const double lnkf = mk->lnA[r] + mk->b[r] * lnT - mk->EaR[r] / T;
    double dG = 0.0;
    for (int g = 0; g < mk->ng[r]; ++g) dG += mk->gnu[r][g] * sGRT[mk->gidx[r][g]][p];
    const double lnKc = -dG + (double)mk->dnu[r] * (mk->ln_p_over_Ru - lnT);
    double fwd = exp(lnkf), rev = exp(lnkf - lnKc);
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const int sf = mk->rf[r][m], sb = mk->rr[r][m];
      if (sf >= 0) fwd *= sConc[sf][p];
      if (sb >= 0) rev *= sConc[sb][p];
    }
    sRate[r][p] = fwd - rev;
  }
  __syncthreads();
  for (int idx = t; idx < NS * NN; idx += kThreads) {
    const int i = idx / NN, p = idx % NN;
    double wdot = 0.0;
    for (int r = 0; r < nr; ++r) {
      const double nu = mk->nud[r][i];
      if (nu != 0.0) wdot += nu * sRate[r][p];
    }
    sS[i][p] = mk->W[i] * wdot;
  }

  // 5. Rusanov total flux f = (g- + g+)/2 - lambda (w+ - w-)/2 at faces e0 + ff; at PE
  //    interfaces the synchronous flux is published and the AT combination is used
  for (int idx = t; idx < V * (TE + 1); idx += kThreads) {
    const int v = idx / (TE + 1), ff = idx % (TE + 1);
    const double wm = sTp[v][ff + 1], wp = sTm[v][ff + 2];
    const double lam = fmax(sLam[0][ff], sLam[1][ff]);
    const double diss = lam * (wp - wm);
    const int i = sI[ff + 1];
    double F;
    if (i >= 0) {
      const double Fs = 0.5 * (sGs[0][v][ff] + sGs[1][v][ff] - diss);
      if (ff < nloc) ring_rec(a.ring, n, a.stage, a.dl.nif, i)[a.ring.off_F + v] = Fs;
      F = sK[ff + 1] > 0 ? sFat[v][ff] : Fs;
    } else {
      F = 0.5 * (sGf[0][v][ff] + sGf[1][v][ff] - diss);
    }
    sF[v][ff] = F;
  }
  __syncthreads();

  // 6. lift, source projection, SSP-RK3 combination
  for (int idx = t; idx < V * M * nloc; idx += kThreads) {
    const int c = idx / nloc, el = idx % nloc;
    const int v = c / M, j = c % M;
    double vol = 0.0, src = 0.0;
#pragma unroll
    for (int qn = 0; qn < Q; ++qn) {
      vol += sWG[qn][j] * sG[v][el * Q + qn];
      if (v >= 3) src += sWB[qn][j] * sS[v >= 3 ? v - 3 : 0][el * Q + qn];
    }
    const double half2j1 = 0.5 * (2 * j + 1);
    const double b = vol - sF[v][el + 1] + ((j & 1) ? -sF[v][el] : sF[v][el]);
    const double L = 2.0 * a.inv_dx * (half2j1 * b) + half2j1 * src;
    const double y = sW[c][el + 2] + a.dt * L;
    const size_t gi = sidx(e0 + el, c, V * M);
    double o;
    if (a.stage == 0) o = y;
    else if (a.stage == 1) o = 0.75 * a.w0[gi] + 0.25 * y;
    else o = (1.0 / 3.0) * a.w0[gi] + (2.0 / 3.0) * y;
    a.wout[gi] = o;
  }
  if (!ok) atomicOr(a.err, (int)kErrState);
  if (a.advance) finish_step(a.step, a.done);
}

// ------------------------------------------------------------------ host side

bool ns_supported(int n_species, int n_reactions) {
  return n_species == kNsMaxSpecies && n_reactions >= 1 && n_reactions <= kNsMaxReactions;
}

adg_status ns_setup(NsArgs &a, const adg_physics *ph, const adg_discretization *d, int E, int M, bool periodic,
                    double dx, const DelayParams &dl, const RingParams &rp, const Tables &tb, const int *face_if,
                    long long *step, unsigned *done, int *err, NsMech *dev_mech) {
  if (!periodic) return ADG_ERR_UNSUPPORTED;
  const adg_mechanism *m = ph->mech;
  if (!ns_supported(m->n_species, m->n_reactions)) return ADG_ERR_UNSUPPORTED;
  NsMech hm;
  std::memset(&hm, 0, sizeof hm);
  hm.ns = m->n_species;
  hm.nr = m->n_reactions;
  hm.Ru = m->Ru;
  hm.p_ref = m->p_ref;
  hm.T_guess = m->T_guess;
  hm.mu_ref = m->mu_ref;
  hm.inv_T_ref = 1.0 / m->T_ref;
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
      hm.nuf[r][i] = f;
      hm.nur[r][i] = b;
      dnu += b - f;
    }
    hm.dnu[r] = dnu;
    int nf = 0, nb = 0, g = 0;
    hm.rf[r][0] = hm.rf[r][1] = hm.rr[r][0] = hm.rr[r][1] = -1;
    for (int i = 0; i < hm.ns; ++i) {
      for (int c = 0; c < hm.nuf[r][i]; ++c) {
        if (nf == 2) return ADG_ERR_UNSUPPORTED;   // at most two reactant molecules
        hm.rf[r][nf++] = i;
      }
      for (int c = 0; c < hm.nur[r][i]; ++c) {
        if (nb == 2) return ADG_ERR_UNSUPPORTED;
        hm.rr[r][nb++] = i;
      }
      const int nu = hm.nur[r][i] - hm.nuf[r][i];
      hm.nud[r][i] = nu;
      if (nu != 0) {
        if (g == 4) return ADG_ERR_UNSUPPORTED;
        hm.gidx[r][g] = i;
        hm.gnu[r][g] = nu;
        ++g;
      }
    }
    hm.ng[r] = g;
  }
  if (hipMemcpy(dev_mech, &hm, sizeof hm, hipMemcpyHostToDevice) != hipSuccess) return ADG_ERR_HIP;
  a.face_if = face_if;
  a.step = step;
  a.done = done;
  a.err = err;
  a.mech = dev_mech;
  a.E = E;
  a.viscous = ph->viscous;
  a.dt = d->dt;
  a.inv_dx = 1.0 / dx;
  a.dl = dl;
  a.ring = rp;
  a.tb = tb;
  (void)M;
  return ADG_OK;
}

template <int M>
static hipError_t ns_M(const NsArgs &a, hipStream_t s) {
  const int blocks = (a.E + kTile - 1) / kTile;
  hipLaunchKernelGGL((ns_stage_kernel<M, kNsMaxSpecies>), dim3(blocks), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_ns_stage(int M, const NsArgs &a, hipStream_t s) {
  switch (M) {
    case 2: return ns_M<2>(a, s);
    case 3: return ns_M<3>(a, s);
    case 4: return ns_M<4>(a, s);
    case 5: return ns_M<5>(a, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace adg
