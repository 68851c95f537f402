// Device code of one time step (Sec. 3.4 order) shared by the two-pass and fused
// schedules: population storage/decoding, the mixture EOS and psi (float64), the
// force stencil, the split and the per-component collision with forcing.
#pragma once
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "lattice.hpp"
#include "lbm.h"

namespace lbmk {

// Per-run constants handed to every kernel by value.
struct KParams {
  int nx, ny, nz, cells;
  int collision, forcing;
  double RT;                       // R * T
  double G, beta, omega;           // omega = 1 / tau
  double aa[LBM_MAX_NC][LBM_MAX_NC];  // sqrt(a_i alpha_i a_j alpha_j)(1 - zeta_ij)
  double b[LBM_MAX_NC];
  double invM[LBM_MAX_NC];
  double gamma[LBM_MAX_NC];
  double s_over_n[LBM_MAX_Q];      // MRT rate / squared norm of each moment row
  double accel[3];
  int* err;                        // device error flag (set to 1 on a domain violation)
};

// ---------------------------------------------------------------------------
// Population storage.  Layout [nc][Q][cells] for the per-direction planes; the
// offset formats add a float base [nc][cells] per cell and component:
//   stored value of direction a at cell y (the post-collision population that
//   streams to y + e_a) = base(y) * (w_a + r_a(y)).
// ---------------------------------------------------------------------------
template <int ST>
struct Pops;

template <>
struct Pops<LBM_F64> {
  using R = double;   // collision arithmetic
  double* f;
  __device__ __forceinline__ double get(int s, int a, int Q, int idx, int cells, double) const {
    return f[(size_t)(s * Q + a) * cells + idx];
  }
  __device__ __forceinline__ void put(int s, int a, int Q, int idx, int cells, double v, double, double) const {
    f[(size_t)(s * Q + a) * cells + idx] = v;
  }
  __device__ __forceinline__ void put_base(int, int, int, double) const {}
};

template <typename H>
struct OffsetPops {
  using R = float;
  float* base;
  H* r;
  __device__ __forceinline__ float get(int s, int a, int Q, int idx, int cells, float w) const {
    return base[(size_t)s * cells + idx] * (w + load(r + (size_t)(s * Q + a) * cells + idx));
  }
  // v: post-collision population; b: the base this cell stores; w: weight of a
  __device__ __forceinline__ void put(int s, int a, int Q, int idx, int cells, float v, float b, float w) const {
    const float rr = (b != 0.0f) ? v / b - w : 0.0f;
    store(r + (size_t)(s * Q + a) * cells + idx, rr);
  }
  __device__ __forceinline__ void put_base(int s, int idx, int cells, float b) const {
    base[(size_t)s * cells + idx] = b;
  }
  static __device__ __forceinline__ float load(const float* p) { return *p; }
  static __device__ __forceinline__ float load(const __half* p) { return __half2float(*p); }
  static __device__ __forceinline__ void store(float* p, float v) { *p = v; }
  static __device__ __forceinline__ void store(__half* p, float v) { *p = __float2half_rn(v); }
};

template <>
struct Pops<LBM_F32_OFS> : OffsetPops<float> {};
template <>
struct Pops<LBM_F16_OFS> : OffsetPops<__half> {};

// Cell coordinates with periodic neighbours.
struct Coord {
  int x, y, z, xm, xp, ym, yp, zm, zp;
  __device__ __forceinline__ int at(int dx, int dy, int dz, int nx, int ny) const {
    const int xx = dx == 0 ? x : (dx > 0 ? xp : xm);
    const int yy = dy == 0 ? y : (dy > 0 ? yp : ym);
    const int zz = dz == 0 ? z : (dz > 0 ? zp : zm);
    return (zz * ny + yy) * nx + xx;
  }
};

__device__ __forceinline__ Coord make_coord(int cell, const KParams& P) {
  Coord c;
  c.x = cell % P.nx;
  const int t = cell / P.nx;
  c.y = t % P.ny;
  c.z = t / P.ny;
  c.xm = c.x == 0 ? P.nx - 1 : c.x - 1;
  c.xp = c.x == P.nx - 1 ? 0 : c.x + 1;
  c.ym = c.y == 0 ? P.ny - 1 : c.y - 1;
  c.yp = c.y == P.ny - 1 ? 0 : c.y + 1;
  c.zm = c.z == 0 ? P.nz - 1 : c.z - 1;
  c.zp = c.z == P.nz - 1 ? 0 : c.z + 1;
  return c;
}

__device__ __forceinline__ void flag_error(const KParams& P) { *P.err = 1; }

// Mixture Peng-Robinson pressure from cell-volume densities (Eq. MCPengRobinson with
// the random mixing rule written in molar densities n_i = rbar_i / M_i:
// b_m rho~ = sum b_i n_i, [a alpha]_m rho~^2 = sum_ij n_i n_j (a alpha)_ij).
template <int NC>
__device__ __forceinline__ double eos_pressure(const KParams& P, const double* rb, double* Bn_out) {
  double n[NC];
  double rt = 0.0, Bn = 0.0;
#pragma unroll
  for (int i = 0; i < NC; ++i) {
    n[i] = rb[i] * P.invM[i];
    rt += n[i];
    Bn += P.b[i] * n[i];
  }
  double An = 0.0;
#pragma unroll
  for (int i = 0; i < NC; ++i) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < NC; ++j) s += P.aa[i][j] * n[j];
    An += n[i] * s;
  }
  *Bn_out = Bn;
  return rt * P.RT / (1.0 - Bn) - An / (1.0 + 2.0 * Bn - Bn * Bn);
}

// psi = sqrt(2 (p_EOS - c_s^2 rho) / (G c_s^2)), Eq. (psicorrected), dt = 1.
template <int NC>
__device__ __forceinline__ double eos_psi(const KParams& P, const double* rb) {
  double Bn;
  const double p = eos_pressure<NC>(P, rb, &Bn);
  double rho = 0.0;
#pragma unroll
  for (int i = 0; i < NC; ++i) rho += rb[i];
  const double X = 6.0 * (p - rho * (1.0 / 3.0)) / P.G;
  if (!(Bn < 1.0) || !(X >= 0.0) || !(X <= 1.0e300)) flag_error(P);
  return sqrt(X);
}

// Equilibrium of Eq. (equilibrium a) for direction a.
template <int LAT, typename R>
__device__ __forceinline__ R feq(int a, R rho, R ux, R uy, R uz, R uu) {
  using V = VS<LAT>;
  const R eu = (R)V::cx(a) * ux + (R)V::cy(a) * uy + (R)V::cz(a) * uz;
  return rho * (R)V::w(a) * ((R)1 + (R)3 * eu + (R)4.5 * eu * eu - (R)1.5 * uu);
}

// Collision with forcing of one component followed by the store of its Q
// post-collision populations at `cell` (pull streaming: the next step reads
// direction a of this cell from the neighbour at cell + e_a).
//   f   : populations of component s at this cell (time t, post-streaming)
//   rs  : rbar_s;  u: shared velocity (Guo: (j+F/2)/rho; EDM: j/rho)
//   Fs  : F_s = chi_s F + rbar_s g (Guo);  du: gamma_s F / Gamma + g (EDM)
template <int LAT, int ST>
__device__ __forceinline__ void collide_store(const KParams& P, const Pops<ST>& out, int s, int cell,
                                              typename Pops<ST>::R* f, double rs_d, const double* u_d,
                                              const double* Fs_d, const double* du_d) {
  using V = VS<LAT>;
  using R = typename Pops<ST>::R;
  constexpr int Q = V::Q;
  const R rs = (R)rs_d;
  const R ux = (R)u_d[0], uy = (R)u_d[1], uz = (R)u_d[2];
  const R uu = ux * ux + uy * uy + uz * uz;
  R fe[Q], src[Q];
  if (P.forcing == LBM_GUO) {
    const R Fx = (R)Fs_d[0], Fy = (R)Fs_d[1], Fz = (R)Fs_d[2];
    const R uF = ux * Fx + uy * Fy + uz * Fz;
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      fe[a] = feq<LAT, R>(a, rs, ux, uy, uz, uu);
      const R cx = (R)V::cx(a), cy = (R)V::cy(a), cz = (R)V::cz(a);
      const R eu = cx * ux + cy * uy + cz * uz;
      const R eF = cx * Fx + cy * Fy + cz * Fz;
      // w_a [ (e_a - u)/cs2 + (e_a.u) e_a / cs4 ] . F_s  (Eq. (equilibrium b) shape)
      src[a] = (R)V::w(a) * ((R)3 * (eF - uF) + (R)9 * eu * eF);
    }
  } else {
    const R vx = ux + (R)du_d[0], vy = uy + (R)du_d[1], vz = uz + (R)du_d[2];
    const R vv = vx * vx + vy * vy + vz * vz;
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      fe[a] = feq<LAT, R>(a, rs, ux, uy, uz, uu);
      src[a] = feq<LAT, R>(a, rs, vx, vy, vz, vv) - fe[a];   // exact-difference term
    }
  }
  R fo[Q];
  if (P.collision == LBM_BGK) {
    const R om = (R)P.omega;
    const R gpre = (P.forcing == LBM_GUO) ? (R)1 - (R)0.5 * om : (R)1;
#pragma unroll
    for (int a = 0; a < Q; ++a) fo[a] = f[a] - om * (f[a] - fe[a]) + gpre * src[a];
  } else {
    // f* = f + src - M^T diag(s_k / |M_k|^2) M (f - feq + h src), h = 1/2 for Guo, 0 for EDM
    const R h = (P.forcing == LBM_GUO) ? (R)0.5 : (R)0;
    R d[Q];
#pragma unroll
    for (int a = 0; a < Q; ++a) d[a] = f[a] - fe[a] + h * src[a];
    R m[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      R acc = 0;
#pragma unroll
      for (int a = 0; a < Q; ++a) {
        const double mk = V::mrow(k, a);
        if (mk != 0.0) acc += (R)mk * d[a];
      }
      m[k] = acc * (R)P.s_over_n[k];
    }
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      R acc = 0;
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        const double mk = V::mrow(k, a);
        if (mk != 0.0) acc += (R)mk * m[k];
      }
      fo[a] = f[a] + src[a] - acc;
    }
  }
  const R base = rs;
  out.put_base(s, cell, P.cells, base);
#pragma unroll
  for (int a = 0; a < Q; ++a) out.put(s, a, Q, cell, P.cells, fo[a], base, (R)V::w(a));
}

// Shared per-cell macroscopic work after the populations are known:
// returns u, Gamma and fills F_s / du for each component.
template <int NC>
__device__ __forceinline__ void cell_forces(const KParams& P, const double* rb, const double* j, const double* F,
                                            double* u, double (*Fs)[3], double (*du)[3]) {
  double rho = 0.0, Gam = 0.0;
#pragma unroll
  for (int s = 0; s < NC; ++s) {
    rho += rb[s];
    Gam += P.gamma[s] * rb[s];
  }
  if (!(Gam > 0.0)) flag_error(P);
  const double g0 = P.accel[0], g1 = P.accel[1], g2 = P.accel[2];
  if (P.forcing == LBM_GUO) {
    u[0] = (j[0] + 0.5 * (F[0] + rho * g0)) / rho;
    u[1] = (j[1] + 0.5 * (F[1] + rho * g1)) / rho;
    u[2] = (j[2] + 0.5 * (F[2] + rho * g2)) / rho;
  } else {
    u[0] = j[0] / rho;
    u[1] = j[1] / rho;
    u[2] = j[2] / rho;
  }
#pragma unroll
  for (int s = 0; s < NC; ++s) {
    const double c = P.gamma[s] / Gam;   // chi_s = gamma_s rbar_s / Gamma
    Fs[s][0] = c * rb[s] * F[0] + rb[s] * g0;
    Fs[s][1] = c * rb[s] * F[1] + rb[s] * g1;
    Fs[s][2] = c * rb[s] * F[2] + rb[s] * g2;
    du[s][0] = c * F[0] + g0;
    du[s][1] = c * F[1] + g1;
    du[s][2] = c * F[2] + g2;
  }
}

}  // namespace lbmk
