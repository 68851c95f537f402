// Velocity sets and orthogonal MRT moment rows for the device kernels.
//
// D2Q9 / D3Q19 with c_s^2 = 1/3 (the paper does not name its set; Sec. 2.1 only
// speaks of weighting factors).  Velocity order (also the order of the population
// planes in memory and of lbm_get_populations):
//   D2Q9 : 0 rest, 1 +x, 2 +y, 3 -x, 4 -y, 5 (+,+), 6 (-,+), 7 (-,-), 8 (+,-)
//   D3Q19: 0 rest, 1..6 faces +x -x +y -y +z -z, 7..10 xy-edges, 11..14 xz-edges,
//          15..18 yz-edges, each edge group (+,+) (-,+) (+,-) (-,-).
// MRT rows: the orthogonal polynomial sets of Lallemand & Luo (D2Q9) and
// d'Humieres et al. (D3Q19), evaluated from their polynomials in (cx, cy, cz).
#pragma once
#include "lbm.h"

namespace lbmk {

template <int LAT>
struct VS;

template <>
struct VS<LBM_D2Q9> {
  static constexpr int D = 2;
  static constexpr int Q = 9;
  __host__ __device__ static constexpr int cx(int a) {
    return (a == 1 || a == 5 || a == 8) ? 1 : ((a == 3 || a == 6 || a == 7) ? -1 : 0);
  }
  __host__ __device__ static constexpr int cy(int a) {
    return (a == 2 || a == 5 || a == 6) ? 1 : ((a == 4 || a == 7 || a == 8) ? -1 : 0);
  }
  __host__ __device__ static constexpr int cz(int) { return 0; }
  __host__ __device__ static constexpr double w(int a) {
    return a == 0 ? 4.0 / 9.0 : (a < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
  }
  // opposite velocity and the first member of each opposite pair
  __host__ __device__ static constexpr int opp(int a) {
    return a == 0 ? 0 : (a < 5 ? (a + 1) % 4 + 1 : (a - 3) % 4 + 5);
  }
  __host__ __device__ static constexpr int pair_first(int p) { return p < 2 ? p + 1 : p + 3; }
  // moment row k evaluated at velocity a
  __host__ __device__ static constexpr double mrow(int k, int a) {
    const double x = cx(a), y = cy(a);
    const double e2 = x * x + y * y;
    switch (k) {
      case 0: return 1.0;
      case 1: return -4.0 + 3.0 * e2;
      case 2: return 4.0 - 10.5 * e2 + 4.5 * e2 * e2;
      case 3: return x;
      case 4: return (-5.0 + 3.0 * e2) * x;
      case 5: return y;
      case 6: return (-5.0 + 3.0 * e2) * y;
      case 7: return x * x - y * y;
      default: return x * y;
    }
  }
};

template <>
struct VS<LBM_D3Q19> {
  static constexpr int D = 3;
  static constexpr int Q = 19;
  __host__ __device__ static constexpr int cx(int a) {
    return (a == 1 || a == 7 || a == 9 || a == 11 || a == 13) ? 1
           : ((a == 2 || a == 8 || a == 10 || a == 12 || a == 14) ? -1 : 0);
  }
  __host__ __device__ static constexpr int cy(int a) {
    return (a == 3 || a == 7 || a == 8 || a == 15 || a == 17) ? 1
           : ((a == 4 || a == 9 || a == 10 || a == 16 || a == 18) ? -1 : 0);
  }
  __host__ __device__ static constexpr int cz(int a) {
    return (a == 5 || a == 11 || a == 12 || a == 15 || a == 16) ? 1
           : ((a == 6 || a == 13 || a == 14 || a == 17 || a == 18) ? -1 : 0);
  }
  __host__ __device__ static constexpr double w(int a) {
    return a == 0 ? 1.0 / 3.0 : (a < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
  }
  // opposite velocity and the first member of each opposite pair
  __host__ __device__ static constexpr int opp(int a) {
    // faces pair as (1,2) (3,4) (5,6); each edge group (+,+)(-,+)(+,-)(-,-) pairs 0<->3, 1<->2
    return a == 0 ? 0 : (a < 7 ? (a % 2 ? a + 1 : a - 1) : (7 + ((a - 7) / 4) * 4 + (3 - (a - 7) % 4)));
  }
  __host__ __device__ static constexpr int pair_first(int p) {
    return p < 3 ? 2 * p + 1 : 7 + ((p - 3) / 2) * 4 + (p - 3) % 2;
  }
  __host__ __device__ static constexpr double mrow(int k, int a) {
    const double x = cx(a), y = cy(a), z = cz(a);
    const double e2 = x * x + y * y + z * z;
    switch (k) {
      case 0: return 1.0;
      case 1: return 19.0 * e2 - 30.0;
      case 2: return (21.0 * e2 * e2 - 53.0 * e2 + 24.0) / 2.0;
      case 3: return x;
      case 4: return (5.0 * e2 - 9.0) * x;
      case 5: return y;
      case 6: return (5.0 * e2 - 9.0) * y;
      case 7: return z;
      case 8: return (5.0 * e2 - 9.0) * z;
      case 9: return 3.0 * x * x - e2;
      case 10: return (3.0 * e2 - 5.0) * (3.0 * x * x - e2);
      case 11: return y * y - z * z;
      case 12: return (3.0 * e2 - 5.0) * (y * y - z * z);
      case 13: return x * y;
      case 14: return y * z;
      case 15: return x * z;
      case 16: return (y * y - z * z) * x;
      case 17: return (z * z - x * x) * y;
      default: return (x * x - y * y) * z;
    }
  }
};

// true if moment row k is odd under velocity reversal (M_k,opp(a) = -M_k,a)
template <int LAT>
__host__ __device__ constexpr bool row_odd_impl(int k) {
  for (int a = 0; a < VS<LAT>::Q; ++a)
    if (VS<LAT>::mrow(k, VS<LAT>::opp(a)) != -VS<LAT>::mrow(k, a)) return false;
  return true;
}

template <int LAT>
__host__ __device__ constexpr double mrow_norm2(int k) {
  double s = 0.0;
  for (int a = 0; a < VS<LAT>::Q; ++a) s += VS<LAT>::mrow(k, a) * VS<LAT>::mrow(k, a);
  return s;
}

template <int LAT>
__host__ __device__ constexpr bool row_odd(int k) { return row_odd_impl<LAT>(k); }

template <int LAT>
__host__ __device__ constexpr int vel(int a, int i) {
  return i == 0 ? VS<LAT>::cx(a) : (i == 1 ? VS<LAT>::cy(a) : VS<LAT>::cz(a));
}

// Row k's moment of the second-order equilibrium feq_a = w_a rho (1 + 3 e.u +
// 9/2 (e.u)^2 - 3/2 u.u), a quadratic in u:
//   sum_a mrow(k, a) feq_a = rho (eq_c0(k) + sum_i eq_c1(k, i) u_i + sum_{i<=j} eq_c2(k, i, j) u_i u_j)
template <int LAT>
__host__ __device__ constexpr double eq_c0(int k) {
  double s = 0.0;
  for (int a = 0; a < VS<LAT>::Q; ++a) s += VS<LAT>::mrow(k, a) * VS<LAT>::w(a);
  return s;
}
template <int LAT>
__host__ __device__ constexpr double eq_c1(int k, int i) {
  double s = 0.0;
  for (int a = 0; a < VS<LAT>::Q; ++a) s += 3.0 * VS<LAT>::mrow(k, a) * VS<LAT>::w(a) * vel<LAT>(a, i);
  return s;
}
template <int LAT>
__host__ __device__ constexpr double eq_c2(int k, int i, int j) {
  double s = 0.0;
  for (int a = 0; a < VS<LAT>::Q; ++a) {
    const double cc = (i == j ? 4.5 : 9.0) * vel<LAT>(a, i) * vel<LAT>(a, j) - (i == j ? 1.5 : 0.0);
    s += VS<LAT>::mrow(k, a) * VS<LAT>::w(a) * cc;
  }
  return s;
}

// squared speed class of velocity a (0 rest, 1 axis, 2 diagonal)
template <int LAT>
__host__ __device__ constexpr int speed2(int a) {
  return VS<LAT>::cx(a) * VS<LAT>::cx(a) + VS<LAT>::cy(a) * VS<LAT>::cy(a) + VS<LAT>::cz(a) * VS<LAT>::cz(a);
}
// row k's entry on speed class c (the entry of the first velocity of that class)
template <int LAT>
__host__ __device__ constexpr double mrow_class(int k, int c) {
  for (int a = 0; a < VS<LAT>::Q; ++a)
    if (speed2<LAT>(a) == c) return VS<LAT>::mrow(k, a);
  return 0.0;
}
// true if row k's entries depend on |e_a|^2 only (the energy rows e and epsilon):
// such a row is a combination of the class sums of the populations
template <int LAT>
__host__ __device__ constexpr bool row_isotropic(int k) {
  for (int a = 0; a < VS<LAT>::Q; ++a)
    if (VS<LAT>::mrow(k, a) != mrow_class<LAT>(k, speed2<LAT>(a))) return false;
  return true;
}

// compile-time checks of the tables: opp is an involution that reverses e_a, the
// pairs cover every moving velocity once, every MRT row is even or odd.
template <int LAT>
constexpr bool tables_consistent() {
  using V = VS<LAT>;
  bool seen[V::Q] = {};
  for (int a = 0; a < V::Q; ++a) {
    const int o = V::opp(a);
    if (V::opp(o) != a || V::cx(o) != -V::cx(a) || V::cy(o) != -V::cy(a) || V::cz(o) != -V::cz(a)) return false;
  }
  for (int p = 0; p < (V::Q - 1) / 2; ++p) {
    const int a = V::pair_first(p), o = V::opp(a);
    if (a == 0 || seen[a] || seen[o]) return false;
    seen[a] = seen[o] = true;
  }
  for (int k = 0; k < V::Q; ++k) {
    bool even = true;
    for (int a = 0; a < V::Q; ++a)
      if (V::mrow(k, V::opp(a)) != V::mrow(k, a)) even = false;
    if (!even && !row_odd<LAT>(k)) return false;
  }
  return true;
}
static_assert(tables_consistent<LBM_D2Q9>(), "D2Q9 tables");
static_assert(tables_consistent<LBM_D3Q19>(), "D3Q19 tables");
// equilibrium moments: density row rho, momentum rows rho u, the energy row e of
// D3Q19 -11 rho + 19 rho u.u, its shear row 3p_xx rho (2u_x^2 - u_y^2 - u_z^2)
constexpr bool near(double a, double b) { return a - b < 1e-12 && b - a < 1e-12; }
static_assert(near(eq_c0<LBM_D3Q19>(0), 1.0) && near(eq_c1<LBM_D3Q19>(3, 0), 1.0) &&
                  near(eq_c1<LBM_D3Q19>(3, 1), 0.0) && near(eq_c0<LBM_D2Q9>(0), 1.0),
              "eq rho, j");
static_assert(near(eq_c0<LBM_D2Q9>(1), -2.0) && near(eq_c2<LBM_D2Q9>(1, 0, 0), 3.0) &&
                  near(eq_c2<LBM_D2Q9>(7, 0, 0), 1.0) && near(eq_c2<LBM_D2Q9>(8, 0, 1), 1.0),
              "eq D2Q9 e, p_xx, p_xy");
static_assert(near(eq_c0<LBM_D3Q19>(1), -11.0) && near(eq_c2<LBM_D3Q19>(1, 0, 0), 19.0) &&
                  near(eq_c2<LBM_D3Q19>(1, 0, 1), 0.0),
              "eq e");
static_assert(near(eq_c2<LBM_D3Q19>(9, 0, 0), 2.0) && near(eq_c2<LBM_D3Q19>(9, 1, 1), -1.0) &&
                  near(eq_c2<LBM_D3Q19>(13, 0, 1), 1.0) && near(eq_c0<LBM_D3Q19>(9), 0.0),
              "eq 3p_xx, p_xy");
static_assert(row_isotropic<LBM_D3Q19>(1) && row_isotropic<LBM_D3Q19>(2) && !row_isotropic<LBM_D3Q19>(9) &&
                  row_isotropic<LBM_D2Q9>(1) && row_isotropic<LBM_D2Q9>(2) && !row_isotropic<LBM_D2Q9>(7),
              "isotropic rows");

}  // namespace lbmk
