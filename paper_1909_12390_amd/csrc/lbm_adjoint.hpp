// Discrete adjoint of one step (BGK or MRT collision, exact-difference or Guo forcing),
// i.e. the transpose of the step's Jacobian applied to the adjoint of the
// post-streaming populations after the step, plus the step's contribution to the
// derivative with respect to the EOS tables (a alpha)_ij (1 - k_ij) and b_i.
//
// Forward step at cell x (post-streaming populations f_sa(x), Sec. 3.4 order):
//   rbar_s = sum_a f_sa, rho = sum_s rbar_s, j = sum_sa e_a f_sa, U = (j + F/2) / rho
//   p = p_EOS(rbar / M) (Eq. MCPengRobinson), X = 6 (p - rho/3) / G, psi = sqrt(X)
//   F(x) = -G sum_a w_a e_a psi(x+e_a) (beta psi(x) + hb psi(x+e_a)),  hb = (1-beta)/2
//   Gamma = sum_s gamma_s rbar_s, X_s = gamma_s F / Gamma (the jump is du_s = X_s + g),
//   w_s = U - X_s/2 (equilibrium velocity), v_s = w_s + du_s = U + X_s/2 + g
//   f*_sa = (1-omega) f_sa + (omega-1) feq_a(rbar_s, w_s) + feq_a(rbar_s, v_s)
//   f_sa(x + e_a, t+1) = f*_sa(x)
// with feq_a(r, v) = w_a r (1 + 3 e.v + 9/2 (e.v)^2 - 3/2 v.v).
//
// Reverse, given h_sa(y) = dL/df_sa(y, t+1):
//   hs_sa(x) = h_sa(x + e_a)                           (adjoint of f*)
//   per component, moments A0 = sum_a w_a hs_a, A1 = sum_a w_a e_a hs_a,
//   A2 = sum_a w_a e_a e_a hs_a give
//     sum_a hs_a feq_a(r, v) = r Phi(v),  Phi(v) = A0 (1 - 3/2 v.v) + 3 A1.v + 9/2 v.A2.v
//     d/dv = r gPhi(v),                   gPhi(v) = -3 A0 v + 3 A1 + 9 A2 v
//   rbar^_s   = (omega-1) Phi_s(w_s) + Phi_s(v_s) + gamma_s Gamma^ - U^.U / rho + [EOS, psi terms]
//   U^        = sum_s rbar_s ((omega-1) gPhi_s(w_s) + gPhi_s(v_s)),  j^ = U^ / rho
//   X^_s      = rbar_s (gPhi_s(v_s) - (omega-1) gPhi_s(w_s)) / 2
//   F^        = sum_s gamma_s X^_s / Gamma + U^ / (2 rho)
//   Gamma^    = -sum_s X_s . X^_s / Gamma
//   psi^(y)   = -G beta sum_a w_a (e_a.F^(y)) psi(y+e_a)
//               - G sum_a w_a (e_a.F^(y-e_a)) (beta psi(y-e_a) + 2 hb psi(y))
//   X^ = psi^ / (2 psi), p^ = 6 X^ / G, rho^ += -2 X^ / G
//   rbar^_s  += p^ dp/dn_s / M_s
//   dL/df_sa(y, t) = (1-omega) hs_sa(y) + e_a.j^(y) + rbar^_s(y)
// and, with n_t = sum n, B = sum b n, A = sum n_i n_j aa_ij, D = 1 + 2B - B^2,
//   dp/dn_i  = RT/(1-B) + n_t RT b_i/(1-B)^2 - 2 (aa n)_i / D + 2 A b_i (1-B) / D^2
//   dp/daa_ij = -n_i n_j / D            dp/db_i = n_i (n_t RT/(1-B)^2 + 2 A (1-B)/D^2).
//
// With Guo forcing (u = (j + F_tot/2)/rho, F_s = gamma_s rbar_s F / Gamma + rbar_s g,
// f*_sa = (1-omega) f_sa + omega feq_a(rbar_s, u) + (1 - omega/2) S_sa,
// S_sa = w_a [3 (e_a - u).F_s + 9 (e_a.u)(e_a.F_s)]) the local part becomes
//   F^_s      = (1 - omega/2) gPhi_s(u)       (sum_a hs_a S_a is linear in F_s)
//   u^        = sum_s [omega rbar_s gPhi_s(u) + (1 - omega/2)(9 A2 F_s - 3 A0 F_s)]
//   F^        = sum_s (gamma_s rbar_s / Gamma) F^_s + u^ / (2 rho)
//   rbar^_s   = omega Phi_s(u) + gamma_s (F^_s.F)/Gamma - gamma_s (sum_t chi_t F^_t.F)/Gamma
//               + F^_s.g - u^.(u - g/2)/rho + [EOS, psi terms]
//
// MRT: f* = feq(u) + (1 - h) src + K (f - feq(u) + h src) with the symmetric
// K = M^-1 (I - S) M = sum_k (1 - s_k)/|M_k|^2 M_k M_k^T (BGK: K = (1 - omega) I).
// With g = K hs the adjoint of f is g (instead of (1 - omega) hs), and every
// equilibrium / source term above takes the moments of the vector that multiplies
// it: EDM  feq(w_s): -g, feq(v_s): hs;   Guo  feq(u): hs - g, src: (hs + g)/2.
//
// Walls (P.bb): the forward pulls with halfway bounce-back, so the adjoint of f*_a(x)
// at a fluid cell is h_{opp(a)}(x) where x + e_a is solid (bit opp(a) of x's mask)
// and h_a(x + e_a) elsewhere; solid cells hold no fluid and a constant psi_w, so
// they carry no adjoint (zero F^, j^, rbar^, output) and no EOS or parameter term.
//
// Two passes per step: ka_cell (everything local to x, writes F^, j^, the local
// part of rbar^ and rbar) and kb_cell (the transposed psi stencil, the EOS adjoint,
// the output and the parameter partials).  psi of the state comes from k_psi.
#pragma once
#include "lbm_aux.hpp"

namespace lbmk {

// Workgroup size of the one-thread-per-cell adjoint kernels: the boxes an adjoint
// runs on are small (C5: 16,384 cells), and 64-thread workgroups spread them over
// four times as many CUs as the step's 256-thread ones (one wavefront per CU on a
// 128^2 box), which shortens these latency-bound kernels.
constexpr int kAdjBlock = 64;
inline int adj_blocks(int cells) { return (int)xcd_grid((unsigned)((cells + kAdjBlock - 1) / kAdjBlock)); }

// per-cell scratch of the adjoint passes (float64, [k][cells])
struct AdjScratch {
  double* Fbar;    // [D]
  double* jbar;    // [D]
  double* rbA;     // [NC] local part of rbar^
  double* rb;      // [NC] rbar of the state
};

// out = K in for the collision operator (BGK: (1 - omega) in; MRT: pair-based
// transform over the rows with (1 - s_k) != 0, as in collide_values)
template <int LAT, int COLL>
__device__ __forceinline__ void apply_K(const KParams& P, const double* in, double* out) {
  using V = VS<LAT>;
  constexpr int Q = V::Q;
  constexpr int NP = (Q - 1) / 2;
  if constexpr (COLL == LBM_BGK) {
    const double k = 1.0 - P.omega;
#pragma unroll
    for (int a = 0; a < Q; ++a) out[a] = k * in[a];
  } else {
    double Sp[NP], Dp[NP], accE[NP], accO[NP], acc0 = 0.0;
    static_for<0, NP>([&](auto Pp) {
      constexpr int p = decltype(Pp)::value;
      constexpr int a = V::pair_first(p), b = V::opp(V::pair_first(p));
      Sp[p] = in[a] + in[b];
      Dp[p] = in[a] - in[b];
      accE[p] = 0.0;
      accO[p] = 0.0;
    });
    // the density row is left out, as in the forward collision (its term vanishes
    // there because sum_a d_a = 0; here its two contributions would cancel)
    static_for<1, Q>([&](auto K) {
      constexpr int k = decltype(K)::value;
      const double ck = P.mrt_c[k];
      double m = 0.0;
      if constexpr (!row_odd<LAT>(k)) {
        if constexpr (V::mrow(k, 0) != 0.0) m += V::mrow(k, 0) * in[0];
        static_for<0, NP>([&](auto Pp) {
          constexpr int p = decltype(Pp)::value;
          constexpr double mk = V::mrow(k, V::pair_first(p));
          if constexpr (mk != 0.0) m += mk * Sp[p];
        });
      } else {
        static_for<0, NP>([&](auto Pp) {
          constexpr int p = decltype(Pp)::value;
          constexpr double mk = V::mrow(k, V::pair_first(p));
          if constexpr (mk != 0.0) m += mk * Dp[p];
        });
      }
      m *= ck;
      if constexpr (!row_odd<LAT>(k) && V::mrow(k, 0) != 0.0) acc0 += V::mrow(k, 0) * m;
      static_for<0, NP>([&](auto Pp) {
        constexpr int p = decltype(Pp)::value;
        constexpr double mk = V::mrow(k, V::pair_first(p));
        if constexpr (mk != 0.0) {
          if constexpr (row_odd<LAT>(k)) accO[p] += mk * m;
          else accE[p] += mk * m;
        }
      });
    });
    out[0] = acc0;
    static_for<0, NP>([&](auto Pp) {
      constexpr int p = decltype(Pp)::value;
      constexpr int a = V::pair_first(p), b = V::opp(V::pair_first(p));
      out[a] = accE[p] + accO[p];
      out[b] = accE[p] - accO[p];
    });
  }
}

// w-weighted moments of a population-shaped vector: A0 = sum w v, A1 = sum w e v,
// A2 = sum w e e v (xx yy zz xy xz yz)
struct WMom {
  double A0, A1[3], A2[6];
};
template <int LAT>
__device__ __forceinline__ WMom wmoments(const double* v) {
  using V = VS<LAT>;
  WMom m = {0.0, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}};
#pragma unroll
  for (int a = 0; a < V::Q; ++a) {
    const double w = V::w(a) * v[a];
    const int ex = V::cx(a), ey = V::cy(a), ez = V::cz(a);
    m.A0 += w;
    if (ex) m.A1[0] += ex * w;
    if (ey) m.A1[1] += ey * w;
    if (ez) m.A1[2] += ez * w;
    if (ex) m.A2[0] += w;
    if (ey) m.A2[1] += w;
    if (ez) m.A2[2] += w;
    if (ex * ey) m.A2[3] += ex * ey * w;
    if (ex * ez) m.A2[4] += ex * ez * w;
    if (ey * ez) m.A2[5] += ey * ez * w;
  }
  return m;
}
__device__ __forceinline__ WMom wcomb(const WMom& a, double ca, const WMom& b, double cb) {
  WMom m;
  m.A0 = ca * a.A0 + cb * b.A0;
#pragma unroll
  for (int d = 0; d < 3; ++d) m.A1[d] = ca * a.A1[d] + cb * b.A1[d];
#pragma unroll
  for (int d = 0; d < 6; ++d) m.A2[d] = ca * a.A2[d] + cb * b.A2[d];
  return m;
}
__device__ __forceinline__ void wA2v(const WMom& m, const double* v, double* out) {
  out[0] = m.A2[0] * v[0] + m.A2[3] * v[1] + m.A2[4] * v[2];
  out[1] = m.A2[3] * v[0] + m.A2[1] * v[1] + m.A2[5] * v[2];
  out[2] = m.A2[4] * v[0] + m.A2[5] * v[1] + m.A2[2] * v[2];
}
// Phi(v) = A0 (1 - 3/2 v.v) + 3 A1.v + 9/2 v.A2.v   (sum_a x_a feq_a(r, v) = r Phi(v))
__device__ __forceinline__ double wphi(const WMom& m, const double* v) {
  double Av[3];
  wA2v(m, v, Av);
  const double vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  return m.A0 * (1.0 - 1.5 * vv) + 3.0 * (m.A1[0] * v[0] + m.A1[1] * v[1] + m.A1[2] * v[2]) +
         4.5 * (v[0] * Av[0] + v[1] * Av[1] + v[2] * Av[2]);
}
// gPhi(v) = d Phi / d v = -3 A0 v + 3 A1 + 9 A2 v
__device__ __forceinline__ void wgphi(const WMom& m, const double* v, double* out) {
  double Av[3];
  wA2v(m, v, Av);
#pragma unroll
  for (int d = 0; d < 3; ++d) out[d] = -3.0 * m.A0 * v[d] + 3.0 * m.A1[d] + 9.0 * Av[d];
}

// The adjoint of the post-collision populations of cell x, one component
// (hs [Q][cells]): h_a(x + e_a), or h_{opp(a)}(x) where x + e_a is solid.
template <int LAT>
__device__ __forceinline__ void gather_h(const double* hs, size_t N, const Coord& c, unsigned cell, unsigned bits,
                                         double* hv) {
  using V = VS<LAT>;
#pragma unroll
  for (int a = 0; a < V::Q; ++a) {
    const bool back = (bits >> V::opp(a)) & 1u;
    hv[a] = back ? hs[(size_t)V::opp(a) * N + cell] : hs[(size_t)a * N + c.at(V::cx(a), V::cy(a), V::cz(a))];
  }
}

template <int LAT, int NC, int ST, int COLL, int FORC>
__global__ __launch_bounds__(kAdjBlock) void ka_cell(KParams P, Pops<ST> state, const double* __restrict__ psi,
                                                 const double* __restrict__ h, AdjScratch S) {
  using V = VS<LAT>;
  using R = typename Pops<ST>::R;
  constexpr int Q = V::Q, D = V::D;
  unsigned cell;
  if (!launch_cell<kAdjBlock>(P, 0, P.nplanes, &cell)) return;
  const Coord c = make_coord(cell, P);
  const size_t N = (size_t)P.cells;
  const unsigned bits = P.bb ? P.bb[cell] : 0u;
  if (bits >> kSolidBit) {          // solid cell: no adjoint
#pragma unroll
    for (int s = 0; s < NC; ++s) {
      S.rbA[(size_t)s * N + cell] = 0.0;
      S.rb[(size_t)s * N + cell] = 0.0;
    }
#pragma unroll
    for (int d = 0; d < D; ++d) {
      S.Fbar[(size_t)d * N + cell] = 0.0;
      S.jbar[(size_t)d * N + cell] = 0.0;
    }
    return;
  }
  // forward quantities at x
  double rb[NC], rho = 0.0, j[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int s = 0; s < NC; ++s) {
    const auto cv = state.comp(s, Q, P.cells);
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      const unsigned nbr = c.at(-V::cx(a), -V::cy(a), -V::cz(a));
      const double v = (double)(P.bb ? pull_bb<LAT>(cv, a, bits, cell, nbr, (R)V::w(a)) : cv.get(a, nbr, (R)V::w(a)));
      acc += v;
      if (V::cx(a)) j[0] += V::cx(a) * v;
      if (V::cy(a)) j[1] += V::cy(a) * v;
      if (V::cz(a)) j[2] += V::cz(a) * v;
    }
    rb[s] = acc;
    rho += acc;
  }
  const double irho = 1.0 / rho;
  double Gam = 0.0;
#pragma unroll
  for (int s = 0; s < NC; ++s) Gam += P.gamma[s] * rb[s];
  const double iG = 1.0 / Gam;
  double F[3];
  force_at<LAT>(P, psi[cell], [&](int a) { return psi[c.at(V::cx(a), V::cy(a), V::cz(a))]; }, F);
  const double* g = P.accel;
  double u[3];   // Guo: (j + F_total/2) / rho;  EDM: U = (j + F/2) / rho
#pragma unroll
  for (int d = 0; d < 3; ++d)
    u[d] = (FORC == LBM_GUO) ? (j[d] + 0.5 * (F[d] + rho * g[d])) * irho : (j[d] + 0.5 * F[d]) * irho;
  double ub[3] = {0.0, 0.0, 0.0}, Fb[3] = {0.0, 0.0, 0.0}, Gb = 0.0;
  double rbA[NC], FbF[NC];
#pragma unroll
  for (int s = 0; s < NC; ++s) {
    // the adjoint of f* (gathered from the downstream neighbours) and K applied to it
    double hv[Q], kv[Q];
    gather_h<LAT>(h + (size_t)s * Q * N, N, c, cell, bits, hv);
    apply_K<LAT, COLL>(P, hv, kv);
    const WMom A = wmoments<LAT>(hv), B = wmoments<LAT>(kv);
    if constexpr (FORC == LBM_EDM) {
      double Xs[3], w[3], v[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        Xs[d] = P.gamma[s] * F[d] * iG;
        w[d] = u[d] - 0.5 * Xs[d];
        v[d] = u[d] + 0.5 * Xs[d] + g[d];
      }
      double gAv[3], gBw[3];
      wgphi(A, v, gAv);
      wgphi(B, w, gBw);
      rbA[s] = wphi(A, v) - wphi(B, w);
      double Xb[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        ub[d] += rb[s] * (gAv[d] - gBw[d]);
        Xb[d] = 0.5 * rb[s] * (gAv[d] + gBw[d]);
        Fb[d] += P.gamma[s] * iG * Xb[d];
      }
      Gb -= (Xs[0] * Xb[0] + Xs[1] * Xb[1] + Xs[2] * Xb[2]) * iG;
      FbF[s] = 0.0;
    } else {
      const WMom E = wcomb(A, 1.0, B, -1.0);     // multiplies feq(u)
      const WMom C = wcomb(A, 0.5, B, 0.5);      // multiplies the source
      const double chi = P.gamma[s] * rb[s] * iG;
      double Fs[3], CF[3], gE[3], gC[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) Fs[d] = chi * F[d] + rb[s] * g[d];
      wA2v(C, Fs, CF);
      wgphi(E, u, gE);
      wgphi(C, u, gC);
      rbA[s] = wphi(E, u);
      double fbs_F = 0.0, fbs_g = 0.0;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double Fbs = gC[d];                  // adjoint of F_s
        ub[d] += rb[s] * gE[d] + (9.0 * CF[d] - 3.0 * C.A0 * Fs[d]);
        Fb[d] += chi * Fbs;
        fbs_F += Fbs * F[d];
        fbs_g += Fbs * g[d];
      }
      rbA[s] += P.gamma[s] * fbs_F * iG + fbs_g;
      FbF[s] = chi * fbs_F;                        // chi_s F^_s . F
    }
  }
  if constexpr (FORC == LBM_GUO) {
    double cs = 0.0;
#pragma unroll
    for (int s = 0; s < NC; ++s) cs += FbF[s];
    Gb = -cs * iG;                                 // d/d Gamma through chi_s = gamma_s rbar_s / Gamma
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) Fb[d] += 0.5 * ub[d] * irho;   // through the F/2 of the velocity
  double uub = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) uub += ub[d] * ((FORC == LBM_GUO) ? (u[d] - 0.5 * g[d]) : u[d]);
  uub *= irho;
#pragma unroll
  for (int s = 0; s < NC; ++s) {
    S.rbA[(size_t)s * N + cell] = rbA[s] + P.gamma[s] * Gb - uub;
    S.rb[(size_t)s * N + cell] = rb[s];
  }
#pragma unroll
  for (int d = 0; d < D; ++d) {
    S.Fbar[(size_t)d * N + cell] = Fb[d];
    S.jbar[(size_t)d * N + cell] = ub[d] * irho;
  }
}

// Parameter partials per block, added to a running per-block accumulator:
// [dL/daa_ij (NC*NC, ordered pairs), dL/db_i (NC)].
template <int LAT, int NC, int COLL>
__global__ __launch_bounds__(kAdjBlock) void kb_cell(KParams P, const double* __restrict__ psi,
                                                 const double* __restrict__ h, AdjScratch S,
                                                 double* __restrict__ hout, double* __restrict__ partials) {
  using V = VS<LAT>;
  constexpr int Q = V::Q, D = V::D, K = NC * NC + NC;
  double vals[K];
#pragma unroll
  for (int k = 0; k < K; ++k) vals[k] = 0.0;
  unsigned cell;
  const bool inside = launch_cell<kAdjBlock>(P, 0, P.nplanes, &cell);
  const unsigned bits = (inside && P.bb) ? P.bb[cell] : 0u;
  if (inside && (bits >> kSolidBit)) {   // solid cell: no adjoint, no EOS or parameter term
    const size_t N = (size_t)P.cells;
#pragma unroll
    for (int s = 0; s < NC; ++s)
#pragma unroll
      for (int a = 0; a < Q; ++a) hout[((size_t)s * Q + a) * N + cell] = 0.0;
  } else if (inside) {
    const Coord c = make_coord(cell, P);
    const size_t N = (size_t)P.cells;
    const double hb = 0.5 * (1.0 - P.beta);
    const double ps = psi[cell];
    // transposed stencil of Eq. (coupledMCforce)
    double pb = 0.0;
    const double Fx = S.Fbar[cell], Fy = S.Fbar[N + cell], Fz = D == 3 ? S.Fbar[2 * N + cell] : 0.0;
#pragma unroll
    for (int a = 1; a < Q; ++a) {
      const int ex = V::cx(a), ey = V::cy(a), ez = V::cz(a);
      const double eF = ex * Fx + ey * Fy + ez * Fz;
      pb += V::w(a) * eF * psi[c.at(ex, ey, ez)] * P.beta;
      const unsigned up = c.at(-ex, -ey, -ez);
      double eFn = ex * S.Fbar[up] + ey * S.Fbar[N + up];
      if (D == 3) eFn += ez * S.Fbar[2 * N + up];
      pb += V::w(a) * eFn * (P.beta * psi[up] + 2.0 * hb * ps);
    }
    pb *= -P.G;
    const double Xb = pb / (2.0 * ps);
    const double pbar = 6.0 * Xb / P.G;
    const double rcommon = -2.0 * Xb / P.G;
    // EOS adjoint
    double n[NC], rt = 0.0, Bn = 0.0;
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      n[i] = S.rb[(size_t)i * N + cell] * P.invM[i];
      rt += n[i];
      Bn += P.b[i] * n[i];
    }
    double an[NC], An = 0.0;
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < NC; ++k) s += P.aa[i][k] * n[k];
      an[i] = s;
      An += n[i] * s;
    }
    const double omB = 1.0 - Bn, iomB = 1.0 / omB;
    const double Dd = 1.0 + 2.0 * Bn - Bn * Bn, iD = 1.0 / Dd;
    const double dpdB = rt * P.RT * iomB * iomB + 2.0 * An * omB * iD * iD;
    double rbar[NC];
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      const double dpdn = P.RT * iomB + P.b[i] * dpdB - 2.0 * an[i] * iD;
      rbar[i] = S.rbA[(size_t)i * N + cell] + rcommon + pbar * dpdn * P.invM[i];
#pragma unroll
      for (int k = 0; k < NC; ++k) vals[i * NC + k] = -pbar * n[i] * n[k] * iD;
      vals[NC * NC + i] = pbar * n[i] * dpdB;
    }
    const double jb[3] = {S.jbar[cell], S.jbar[N + cell], D == 3 ? S.jbar[2 * N + cell] : 0.0};
#pragma unroll
    for (int s = 0; s < NC; ++s) {
      double* ho = hout + (size_t)s * Q * N;
      double hv[Q], kv[Q];
      gather_h<LAT>(h + (size_t)s * Q * N, N, c, cell, bits, hv);
      apply_K<LAT, COLL>(P, hv, kv);
#pragma unroll
      for (int a = 0; a < Q; ++a) {
        const double ej = V::cx(a) * jb[0] + V::cy(a) * jb[1] + V::cz(a) * jb[2];
        ho[(size_t)a * N + cell] = kv[a] + ej + rbar[s];
      }
    }
  }
  block_partials_add<K, kAdjBlock>(vals, partials);
}

// Masked molar sums N_s = sum_{mask} rbar_s / M_s of the post-streaming state
// (per-block partials, [NC]).
template <int LAT, int NC, int ST>
__global__ __launch_bounds__(kAdjBlock) void k_masked_moles(KParams P, Pops<ST> state,
                                                        const unsigned char* __restrict__ mask,
                                                        double* __restrict__ partials) {
  double vals[NC];
#pragma unroll
  for (int s = 0; s < NC; ++s) vals[s] = 0.0;
  unsigned cell;
  if (launch_cell<kAdjBlock>(P, 0, P.nplanes, &cell) && mask[cell]) {
    const unsigned bits = P.bb ? P.bb[cell] : 0u;
    if (!(bits >> kSolidBit)) {         // solid cells hold no fluid
      const Coord c = make_coord(cell, P);
      typename Pops<ST>::R jr[3] = {0, 0, 0};
#pragma unroll
      for (int s = 0; s < NC; ++s) vals[s] = pull_moments<LAT, ST>(P, state, s, c, jr, cell, bits) * P.invM[s];
    }
  }
  block_partials<NC, kAdjBlock, false>(vals, partials);   // block-major, for k_accumulate
}

// Adjoint seed of L(N): dL/df_sa(y) = mask(y) * coef_s for every direction.
template <int LAT, int NC>
__global__ __launch_bounds__(kAdjBlock) void k_adj_seed(KParams P, const unsigned char* __restrict__ mask,
                                                    double c0, double c1, double c2, double c3,
                                                    double* __restrict__ h) {
  using V = VS<LAT>;
  unsigned cell;
  if (!launch_cell<kAdjBlock>(P, 0, P.nplanes, &cell)) return;
  const double coef[4] = {c0, c1, c2, c3};
  const size_t N = (size_t)P.cells;
  const bool in = mask[cell] != 0;
#pragma unroll
  for (int s = 0; s < NC; ++s)
#pragma unroll
    for (int a = 0; a < V::Q; ++a) h[((size_t)s * V::Q + a) * N + cell] = in ? coef[s] : 0.0;
}

}  // namespace lbmk
