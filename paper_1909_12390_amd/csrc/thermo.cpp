// Host float64 Peng-Robinson mixture thermodynamics behind the C ABI
// (lbm_critical, lbm_fugacity, lbm_flash, lbm_bubble_pressure, lbm_dew_pressure).
//
// Paper: Sec. 3.2 (Eqs. MCPengRobinson, randommixingrule, PRcubic, cubiccoeff,
// fugacity, fugacitycoeff2, solutionselection, error) and Sec. 3.1 Eq. (gamma).
// Readings of the printed equations (shared with the model description):
//   * cubic in Z: Z^3 + (B-1)Z^2 + (A - 3B^2 - 2B)Z - (AB - B^2 - B^3) = 0, the
//     polynomial the EOS itself produces with Z = p/(rho~ R T);
//   * A_ij = sqrt(a_i alpha_i a_j alpha_j)(1 - zeta_ij) p/(RT)^2, B_i = b_i p/(RT)
//     (reduced form: Omega_a alpha_i p_ri / T_ri^2 and Omega_b p_ri / T_ri);
//   * flash: Wilson start, successive substitution on ln K, Rachford-Rice solved by
//     Newton safeguarded with bisection on its pole-free bracket.
#include "lbm.h"
#include "lbm_internal.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace {

constexpr double kOmegaA = 0.45724;
constexpr double kOmegaB = 0.0778;
constexpr double kSqrt2 = 1.41421356237309504880;

struct Mix {
  int nc;
  double R;
  double a[LBM_MAX_NC], b[LBM_MAX_NC], w[LBM_MAX_NC], M[LBM_MAX_NC];
  double k[LBM_MAX_NC][LBM_MAX_NC];
  double Tc[LBM_MAX_NC], pc[LBM_MAX_NC], m[LBM_MAX_NC];
};

bool load_mix(const lbm_mixture* in, Mix* mx) {
  if (!in) return lbm_fail(LBM_ERR_ARG, "mixture is NULL"), false;
  if (in->nc < 1 || in->nc > LBM_MAX_NC) return lbm_fail(LBM_ERR_ARG, "nc must be 1..4"), false;
  if (!(in->R > 0)) return lbm_fail(LBM_ERR_ARG, "R must be positive"), false;
  mx->nc = in->nc;
  mx->R = in->R;
  for (int i = 0; i < in->nc; ++i) {
    if (!(in->a[i] > 0) || !(in->b[i] > 0) || !(in->M[i] > 0))
      return lbm_fail(LBM_ERR_ARG, "a_i, b_i, M_i must be positive"), false;
    mx->a[i] = in->a[i];
    mx->b[i] = in->b[i];
    mx->w[i] = in->omega[i];
    mx->M[i] = in->M[i];
    for (int j = 0; j < in->nc; ++j) mx->k[i][j] = in->k[i][j];
    // Sec. 3.2: a = Omega_a R^2 Tc^2 / pc, b = Omega_b R Tc / pc  =>  Tc, pc
    mx->Tc[i] = kOmegaB * in->a[i] / (kOmegaA * in->b[i] * in->R);
    mx->pc[i] = kOmegaB * in->R * mx->Tc[i] / in->b[i];
    const double om = in->omega[i];
    mx->m[i] = (om <= 0.49) ? 0.374640 + om * (1.54226 - 0.26992 * om)
                            : 0.379642 + om * (1.48503 + om * (-0.164423 + 0.016666 * om));
  }
  return true;
}

// a_i alpha_i(T)
void aalpha(const Mix& mx, double T, double* aa) {
  for (int i = 0; i < mx.nc; ++i) {
    const double s = 1.0 + mx.m[i] * (1.0 - std::sqrt(T / mx.Tc[i]));
    aa[i] = mx.a[i] * s * s;
  }
}

// Dimensionless A_ij and B_i at (T, p) and the mixture A, B at composition c.
struct PhaseCoef {
  double Aij[LBM_MAX_NC][LBM_MAX_NC];
  double Bi[LBM_MAX_NC];
  double A, B;
};

void phase_coef(const Mix& mx, double T, double p, const double* c, PhaseCoef* pc) {
  double aa[LBM_MAX_NC];
  aalpha(mx, T, aa);
  const double RT = mx.R * T;
  const double sa = p / (RT * RT), sb = p / RT;
  pc->A = 0.0;
  pc->B = 0.0;
  for (int i = 0; i < mx.nc; ++i) {
    pc->Bi[i] = mx.b[i] * sb;
    pc->B += c[i] * pc->Bi[i];
    for (int j = 0; j < mx.nc; ++j) {
      pc->Aij[i][j] = std::sqrt(aa[i] * aa[j]) * (1.0 - mx.k[i][j]) * sa;
      pc->A += c[i] * c[j] * pc->Aij[i][j];
    }
  }
}

// Real roots of Z^3 + c2 Z^2 + c1 Z + c0 (trigonometric / Cardano), Newton-polished.
int cubic_real_roots(double c2, double c1, double c0, double* r) {
  const double q = (3.0 * c1 - c2 * c2) / 9.0;
  const double rr = (9.0 * c2 * c1 - 27.0 * c0 - 2.0 * c2 * c2 * c2) / 54.0;
  const double disc = q * q * q + rr * rr;
  int n = 0;
  if (disc < 0.0) {
    const double th = std::acos(std::max(-1.0, std::min(1.0, rr / std::sqrt(-q * q * q))));
    const double s = 2.0 * std::sqrt(-q);
    r[0] = s * std::cos(th / 3.0) - c2 / 3.0;
    r[1] = s * std::cos((th + 2.0 * M_PI) / 3.0) - c2 / 3.0;
    r[2] = s * std::cos((th + 4.0 * M_PI) / 3.0) - c2 / 3.0;
    n = 3;
  } else {
    const double sd = std::sqrt(disc);
    r[0] = std::cbrt(rr + sd) + std::cbrt(rr - sd) - c2 / 3.0;
    n = 1;
  }
  for (int i = 0; i < n; ++i) {
    double z = r[i];
    for (int it = 0; it < 6; ++it) {
      const double f = ((z + c2) * z + c1) * z + c0;
      const double d = (3.0 * z + 2.0 * c2) * z + c1;
      if (d == 0.0) break;
      const double dz = f / d;
      z -= dz;
      if (std::fabs(dz) <= 1e-16 * std::fabs(z)) break;
    }
    r[i] = z;
  }
  std::sort(r, r + n);
  return n;
}

// Roots above B of the PR cubic, ascending.
int pr_roots(double A, double B, double* z) {
  double r[3];
  const int n = cubic_real_roots(B - 1.0, A - 3.0 * B * B - 2.0 * B, -(A * B - B * B - B * B * B), r);
  int m = 0;
  for (int i = 0; i < n; ++i)
    if (r[i] > B) z[m++] = r[i];
  return m;
}

// ln phi_i, Eq. (fugacitycoeff2).
void ln_phi(const Mix& mx, const PhaseCoef& pc, double Z, const double* c, double* out) {
  const double L = std::log((Z + (1.0 - kSqrt2) * pc.B) / (Z + (1.0 + kSqrt2) * pc.B));
  const double lzb = std::log(Z - pc.B);
  const double pre = pc.A / (2.0 * kSqrt2 * pc.B);
  for (int i = 0; i < mx.nc; ++i) {
    double s = 0.0;
    for (int j = 0; j < mx.nc; ++j) s += pc.Aij[i][j] * c[j];
    const double bb = pc.Bi[i] / pc.B;
    out[i] = -lzb + bb * (Z - 1.0) + pre * (2.0 * s / pc.A - bb) * L;
  }
}

// Gibbs-energy difference G(Zmax) - G(Zmin) over RT, Eq. (solutionselection).
double dG(double zmax, double zmin, double A, double B) {
  const double s1 = 1.0 + kSqrt2, s2 = 1.0 - kSqrt2;
  return (zmax - zmin) + std::log((zmin - B) / (zmax - B)) +
         A / (2.0 * kSqrt2 * B) * std::log(((zmin + s1 * B) * (zmax + s2 * B)) / ((zmin + s2 * B) * (zmax + s1 * B)));
}

// Z of a phase of composition c at (T, p) with the Gibbs root choice, and ln phi.
bool phase(const Mix& mx, double T, double p, const double* c, double* Z, double* lphi) {
  PhaseCoef pc;
  phase_coef(mx, T, p, c, &pc);
  double z[3];
  const int n = pr_roots(pc.A, pc.B, z);
  if (n == 0) return false;
  double zz = z[0];
  if (n > 1) zz = (dG(z[n - 1], z[0], pc.A, pc.B) >= 0.0) ? z[0] : z[n - 1];
  *Z = zz;
  ln_phi(mx, pc, zz, c, lphi);
  return true;
}

// Rachford-Rice: sum z_i (K_i - 1) / (1 + V (K_i - 1)) = 0 on (1/(1-Kmax), 1/(1-Kmin)).
bool rachford_rice(int nc, const double* z, const double* K, double* V) {
  double kmax = K[0], kmin = K[0];
  for (int i = 1; i < nc; ++i) {
    kmax = std::max(kmax, K[i]);
    kmin = std::min(kmin, K[i]);
  }
  if (!(kmax > 1.0 && kmin < 1.0)) return false;
  double lo = 1.0 / (1.0 - kmax), hi = 1.0 / (1.0 - kmin);
  double v = 0.5 * (lo + hi);
  for (int it = 0; it < 200; ++it) {
    double g = 0.0, dg = 0.0;
    for (int i = 0; i < nc; ++i) {
      const double km = K[i] - 1.0;
      const double den = 1.0 + v * km;
      g += z[i] * km / den;
      dg -= z[i] * km * km / (den * den);
    }
    if (g > 0.0) lo = v; else hi = v;
    double vn = v - g / dg;
    if (!(vn > lo && vn < hi)) vn = 0.5 * (lo + hi);
    if (std::fabs(vn - v) <= 1e-16 * std::max(1.0, std::fabs(v)) || hi - lo <= 1e-16 * std::max(1.0, std::fabs(v))) {
      v = vn;
      break;
    }
    v = vn;
  }
  *V = v;
  return true;
}

void wilson(const Mix& mx, double T, double p, double* K) {
  for (int i = 0; i < mx.nc; ++i)
    K[i] = mx.pc[i] / p * std::exp(5.373 * (1.0 + mx.w[i]) * (1.0 - mx.Tc[i] / T));
}

}  // namespace

extern "C" lbm_status lbm_critical(const lbm_mixture* mix, double* Tc, double* pc) {
  Mix mx;
  if (!load_mix(mix, &mx)) return LBM_ERR_ARG;
  for (int i = 0; i < mx.nc; ++i) {
    if (Tc) Tc[i] = mx.Tc[i];
    if (pc) pc[i] = mx.pc[i];
  }
  return LBM_OK;
}

extern "C" lbm_status lbm_fugacity(const lbm_mixture* mix, double T, int nstates, const double* n,
                                   double* p_out, double* Z_out, double* lnphi_out, double* fug_out) {
  Mix mx;
  if (!load_mix(mix, &mx)) return LBM_ERR_ARG;
  if (nstates < 0 || (nstates > 0 && !n) || !(T > 0)) return lbm_fail(LBM_ERR_ARG, "bad fugacity arguments");
  double aa[LBM_MAX_NC];
  aalpha(mx, T, aa);
  const int nc = mx.nc;
  for (int s = 0; s < nstates; ++s) {
    const double* ns = n + (size_t)s * nc;
    double rt = 0.0, Bn = 0.0, An = 0.0;
    for (int i = 0; i < nc; ++i) {
      rt += ns[i];
      Bn += mx.b[i] * ns[i];
    }
    for (int i = 0; i < nc; ++i)
      for (int j = 0; j < nc; ++j) An += ns[i] * ns[j] * std::sqrt(aa[i] * aa[j]) * (1.0 - mx.k[i][j]);
    if (!(rt > 0) || !(Bn < 1.0)) return lbm_fail(LBM_ERR_DOMAIN, "state %d outside the EOS domain", s);
    // Eq. (MCPengRobinson) written with molar densities n_i = c_i rho~
    const double p = rt * mx.R * T / (1.0 - Bn) - An / (1.0 + 2.0 * Bn - Bn * Bn);
    const double Z = p / (rt * mx.R * T);
    double c[LBM_MAX_NC], lp[LBM_MAX_NC];
    for (int i = 0; i < nc; ++i) c[i] = ns[i] / rt;
    if (p_out) p_out[s] = p;
    if (Z_out) Z_out[s] = Z;
    if (lnphi_out || fug_out) {
      if (!(p > 0)) return lbm_fail(LBM_ERR_DOMAIN, "state %d has p <= 0; fugacity undefined", s);
      PhaseCoef pc;
      phase_coef(mx, T, p, c, &pc);
      ln_phi(mx, pc, Z, c, lp);
      for (int i = 0; i < nc; ++i) {
        if (lnphi_out) lnphi_out[(size_t)s * nc + i] = lp[i];
        if (fug_out) fug_out[(size_t)s * nc + i] = std::exp(lp[i]) * c[i] * p;  // Eq. (fugacity)
      }
    }
  }
  return LBM_OK;
}

extern "C" lbm_status lbm_flash(const lbm_mixture* mix, double T, double p, const double* z, lbm_flash_result* out) {
  Mix mx;
  if (!load_mix(mix, &mx)) return LBM_ERR_ARG;
  if (!z || !out || !(T > 0) || !(p > 0)) return lbm_fail(LBM_ERR_ARG, "bad flash arguments");
  const int nc = mx.nc;
  double zs = 0.0;
  for (int i = 0; i < nc; ++i) {
    if (!(z[i] > 0)) return lbm_fail(LBM_ERR_ARG, "z_i must be positive");
    zs += z[i];
  }
  double zz[LBM_MAX_NC], K[LBM_MAX_NC], lnK[LBM_MAX_NC], x[LBM_MAX_NC], y[LBM_MAX_NC];
  double lpl[LBM_MAX_NC], lpv[LBM_MAX_NC], Zl = 0, Zv = 0, V = 0;
  for (int i = 0; i < nc; ++i) zz[i] = z[i] / zs;
  wilson(mx, T, p, K);
  for (int i = 0; i < nc; ++i) lnK[i] = std::log(K[i]);
  int it = 0;
  bool conv = false;
  auto split = [&](double v) {
    double sx = 0.0, sy = 0.0;
    for (int i = 0; i < nc; ++i) {
      x[i] = zz[i] / (1.0 + v * (K[i] - 1.0));
      y[i] = K[i] * x[i];
      sx += x[i];
      sy += y[i];
    }
    for (int i = 0; i < nc; ++i) {
      x[i] /= sx;
      y[i] /= sy;
    }
  };
  for (it = 1; it <= 20000; ++it) {
    if (!rachford_rice(nc, zz, K, &V)) return lbm_fail(LBM_ERR_SINGLEPHASE, "flash: K values do not bracket 1");
    split(V);
    if (!phase(mx, T, p, x, &Zl, lpl) || !phase(mx, T, p, y, &Zv, lpv))
      return lbm_fail(LBM_ERR_NOCONVERGE, "flash: no EOS root");
    double dmax = 0.0, kmax = 0.0;
    for (int i = 0; i < nc; ++i) {
      const double nk = lpl[i] - lpv[i];
      dmax = std::max(dmax, std::fabs(nk - lnK[i]));
      kmax = std::max(kmax, std::fabs(nk));
      lnK[i] = nk;
      K[i] = std::exp(nk);
    }
    if (kmax < 1e-6) return lbm_fail(LBM_ERR_SINGLEPHASE, "flash: trivial solution");
    if (dmax < 1e-13) {
      conv = true;
      break;
    }
  }
  if (!conv) return lbm_fail(LBM_ERR_NOCONVERGE, "flash: successive substitution did not converge");
  if (!rachford_rice(nc, zz, K, &V)) return lbm_fail(LBM_ERR_SINGLEPHASE, "flash: K values do not bracket 1");
  if (!(V > 0.0 && V < 1.0)) return lbm_fail(LBM_ERR_SINGLEPHASE, "flash: vapor fraction %g outside (0,1)", V);
  split(V);
  if (!phase(mx, T, p, x, &Zl, lpl) || !phase(mx, T, p, y, &Zv, lpv))
    return lbm_fail(LBM_ERR_NOCONVERGE, "flash: no EOS root");
  std::memset(out, 0, sizeof(*out));
  out->V = V;
  out->Zl = Zl;
  out->Zv = Zv;
  out->rho_l = p / (Zl * mx.R * T);
  out->rho_v = p / (Zv * mx.R * T);
  out->iterations = it;
  int ref = 0;
  double res = 0.0;
  for (int i = 0; i < nc; ++i) {
    out->x[i] = x[i];
    out->y[i] = y[i];
    out->K[i] = y[i] / x[i];
    out->rbar_l[i] = out->rho_l * x[i] * mx.M[i];  // Sec. 2.2 relation, molar form
    out->rbar_v[i] = out->rho_v * y[i] * mx.M[i];
    out->fug_l[i] = std::exp(lpl[i]) * x[i] * p;
    out->fug_v[i] = std::exp(lpv[i]) * y[i] * p;
    const double q = out->fug_l[i] / out->fug_v[i] - 1.0;  // Eq. (error)
    res += q * q;
    if (out->K[i] < out->K[ref]) ref = i;
  }
  out->residual = res;
  // Eq. (gamma): least volatile component (smallest K) is the reference with gamma = 1
  const double lref = std::log(out->rbar_l[ref] / out->rbar_v[ref]);
  for (int i = 0; i < nc; ++i) out->gamma[i] = (i == ref) ? 1.0 : std::log(out->rbar_l[i] / out->rbar_v[i]) / lref;
  return LBM_OK;
}

namespace {
// Saturation pressure with one phase fixed at composition z and an incipient phase.
// bubble: liquid = z; p <- p * sum K z.  dew: vapor = z; p <- p / sum z / K.
lbm_status saturation(const lbm_mixture* mix, double T, const double* z, bool bubble, double* p_out) {
  Mix mx;
  if (!load_mix(mix, &mx)) return LBM_ERR_ARG;
  if (!z || !p_out || !(T > 0)) return lbm_fail(LBM_ERR_ARG, "bad saturation arguments");
  const int nc = mx.nc;
  double zz[LBM_MAX_NC], K[LBM_MAX_NC], w[LBM_MAX_NC], lp1[LBM_MAX_NC], lp2[LBM_MAX_NC], Z;
  double zs = 0.0;
  for (int i = 0; i < nc; ++i) zs += z[i];
  for (int i = 0; i < nc; ++i) zz[i] = z[i] / zs;
  double p;
  wilson(mx, T, 1.0, K);  // K at unit pressure, scaled below
  if (bubble) {
    p = 0.0;
    for (int i = 0; i < nc; ++i) p += zz[i] * K[i];
  } else {
    double s = 0.0;
    for (int i = 0; i < nc; ++i) s += zz[i] / K[i];
    p = 1.0 / s;
  }
  wilson(mx, T, p, K);
  for (int it = 0; it < 20000; ++it) {
    double sw = 0.0;
    for (int i = 0; i < nc; ++i) {
      w[i] = bubble ? K[i] * zz[i] : zz[i] / K[i];
      sw += w[i];
    }
    for (int i = 0; i < nc; ++i) w[i] /= sw;
    const double* liq = bubble ? zz : w;
    const double* vap = bubble ? w : zz;
    if (!phase(mx, T, p, liq, &Z, lp1) || !phase(mx, T, p, vap, &Z, lp2))
      return lbm_fail(LBM_ERR_NOCONVERGE, "saturation: no EOS root");
    double S = 0.0;
    for (int i = 0; i < nc; ++i) {
      K[i] = std::exp(lp1[i] - lp2[i]);
      S += bubble ? K[i] * zz[i] : zz[i] / K[i];
    }
    const double pn = bubble ? p * S : p / S;
    if (!(pn > 0) || !std::isfinite(pn)) return lbm_fail(LBM_ERR_NOCONVERGE, "saturation: pressure diverged");
    if (std::fabs(S - 1.0) < 1e-13) {
      *p_out = pn;
      return LBM_OK;
    }
    p = pn;
  }
  return lbm_fail(LBM_ERR_NOCONVERGE, "saturation pressure did not converge");
}
}  // namespace

extern "C" lbm_status lbm_bubble_pressure(const lbm_mixture* mix, double T, const double* z, double* p_out) {
  return saturation(mix, T, z, true, p_out);
}

extern "C" lbm_status lbm_dew_pressure(const lbm_mixture* mix, double T, const double* z, double* p_out) {
  return saturation(mix, T, z, false, p_out);
}

void lbm_internal_aalpha(const lbm_mixture* mix, double T, double* aa_out) {
  Mix mx;
  if (!load_mix(mix, &mx)) return;
  aalpha(mx, T, aa_out);
}

// Chain rule from the EOS tables to the component parameters.  With
// (a alpha)_l = a_l alpha_l(T / Tc_l), Tc_l = (Omega_b / Omega_a) a_l / (b_l R) and
// aa_ij = sqrt((a alpha)_i (a alpha)_j) (1 - k_ij) (Sec. 3.2):
//   d aa_ij / d (a alpha)_l = aa_ij (d_il + d_jl) / (2 (a alpha)_l)
//   d (a alpha)_l / d a_l = alpha_l + Tc_l alpha'_l,  d (a alpha)_l / d b_l = -a_l Tc_l alpha'_l / b_l
//   alpha'_l = d alpha_l / d Tc_l = sqrt(alpha_l) m_l sqrt(T / Tc_l) / Tc_l
//   d aa_ij / d k_ij = -sqrt((a alpha)_i (a alpha)_j) for each ordered pair.
extern "C" lbm_status lbm_eos_param_grad(const lbm_mixture* mix, double T, const double* d_aa,
                                         const double* d_b_direct, double* d_k, double* d_a, double* d_b) {
  Mix mx;
  if (!load_mix(mix, &mx)) return LBM_ERR_ARG;
  if (!d_aa || !d_b_direct || !d_k || !d_a || !d_b) return lbm_fail(LBM_ERR_ARG, "NULL argument");
  if (!(T > 0.0)) return lbm_fail(LBM_ERR_ARG, "T must be positive");
  const int nc = mx.nc;
  double al[LBM_MAX_NC], aal[LBM_MAX_NC], dal[LBM_MAX_NC];
  for (int l = 0; l < nc; ++l) {
    const double r = std::sqrt(T / mx.Tc[l]);
    const double s = 1.0 + mx.m[l] * (1.0 - r);
    al[l] = s * s;
    aal[l] = mx.a[l] * al[l];
    dal[l] = s * mx.m[l] * r / mx.Tc[l];
  }
  for (int l = 0; l < nc; ++l) {
    double g = 0.0;
    for (int j = 0; j < nc; ++j) {
      const double aa_lj = std::sqrt(aal[l] * aal[j]) * (1.0 - mx.k[l][j]);
      const double aa_jl = std::sqrt(aal[j] * aal[l]) * (1.0 - mx.k[j][l]);
      g += d_aa[l * nc + j] * aa_lj + d_aa[j * nc + l] * aa_jl;
    }
    g /= 2.0 * aal[l];
    d_a[l] = g * (al[l] + mx.Tc[l] * dal[l]);
    d_b[l] = d_b_direct[l] - g * mx.a[l] * mx.Tc[l] * dal[l] / mx.b[l];
  }
  for (int i = 0; i < nc; ++i)
    for (int j = 0; j < nc; ++j)
      d_k[i * nc + j] = (i == j) ? 0.0 : -std::sqrt(aal[i] * aal[j]) * (d_aa[i * nc + j] + d_aa[j * nc + i]);
  return LBM_OK;
}
