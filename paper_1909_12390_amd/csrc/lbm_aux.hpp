// Kernels around the step: macroscopic fields with per-block partial sums for the
// conservation totals, and import / export / equilibrium initialisation of the
// population state (pull layout: the stored direction a at cell y is the
// population that arrives at y + e_a).
#pragma once
#include "lbm_kernels.hpp"

namespace lbmk {

// Butterfly sums over the wavefront of K values at once (every lane ends with the
// totals): each step exchanges all K values before adding, so the K exchanges of a
// step are in flight together (one wait per step rather than one per value)
template <int K>
__device__ __forceinline__ void wave_sums(double* v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    double t[K];
#pragma unroll
    for (int k = 0; k < K; ++k) t[k] = __shfl_xor(v[k], off, 64);
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] += t[k];
  }
}

// The block's sums of vals[0..K) into partials[k][block] (ByTotal: total-major over
// gridDim.x blocks, so that the moments' final pass reads each total's partials
// contiguously) or partials[block][k] (block-major, read by the adjoint's
// accumulator pass, k_accumulate).
template <int K, int B = kBlock, bool ByTotal = true>   // B: threads per workgroup
__device__ __forceinline__ void block_partials(double* vals, double* partials) {
  __shared__ double red[B / 64][K];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  wave_sums<K>(vals);
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (lane == 0) red[wv][k] = vals[k];
  __syncthreads();
  if (threadIdx.x < K) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < B / 64; ++w) s += red[w][threadIdx.x];
    if constexpr (ByTotal) partials[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = s;
    else partials[(size_t)blockIdx.x * K + threadIdx.x] = s;
  }
}

// the block's sums of vals[0..K) added to partials[block][k] (block-major: a running
// per-block accumulator across launches on one stream; each block owns its row)
template <int K, int B = kBlock>
__device__ __forceinline__ void block_partials_add(double* vals, double* partials) {
  __shared__ double red[B / 64][K];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  wave_sums<K>(vals);
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (lane == 0) red[wv][k] = vals[k];
  __syncthreads();
  if (threadIdx.x < K) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < B / 64; ++w) s += red[w][threadIdx.x];
    partials[(size_t)blockIdx.x * K + threadIdx.x] += s;
  }
}

// rbar_s, u = (j + F_total/2)/rho, p_EOS and psi of every cell; per-block partial
// sums of [mass_s (nc), momentum (D), force (D), number of fluid cells with
// rbar_s < 0 (nc)] in a fixed order.  The scheme does not keep the partial
// densities positive (nothing is clamped); the counts report where a trace
// component has crossed zero.
template <int LAT, int NC, int ST>
__global__ __launch_bounds__(kBlock) void k_moments(KParams P, Pops<ST> in, const double* __restrict__ psi,
                                                   double* rho_out, double* u_out, double* p_out, double* psi_out,
                                                   double* partials) {
  using V = VS<LAT>;
  using R = typename Pops<ST>::R;
  constexpr int D = V::D, K = 2 * NC + 2 * D;
  double vals[K];
#pragma unroll
  for (int k = 0; k < K; ++k) vals[k] = 0.0;
  unsigned cell;
  const bool inside = launch_cell(P, 0, P.nplanes, &cell);
  const unsigned bits = (inside && P.bb) ? P.bb[cell] : 0u;
  if (inside && (bits >> kSolidBit)) {   // solid cell: no fluid; psi is the wall's
    if (rho_out)
#pragma unroll
      for (int s = 0; s < NC; ++s) rho_out[(size_t)s * P.cells + cell] = 0.0;
    if (u_out)
#pragma unroll
      for (int d = 0; d < D; ++d) u_out[(size_t)d * P.cells + cell] = 0.0;
    if (p_out) p_out[cell] = 0.0;
    if (psi_out) psi_out[cell] = psi[cell];
  } else if (inside) {
    const Coord c = make_coord(cell, P);
    double rb[NC], rho = 0.0;
    R jr[3] = {0, 0, 0};
    if constexpr (ST == LBM_F64) {
#pragma unroll
      for (int s = 0; s < NC; ++s) {
        rb[s] = pull_moments<LAT, ST>(P, in, s, c, jr, cell, bits);
        rho += rb[s];
      }
    } else {   // every component of a direction by one vector load (ilv_pull_cell)
      using H = typename Pops<ST>::Elem;
      float f[NC][V::Q];
      ilv_pull_cell<LAT, NC, H, kPopLoad>(IlvBufs<H, NC, V::Q>(in, P.cells), c, cell, bits, P.bb != nullptr, f);
#pragma unroll
      for (int s = 0; s < NC; ++s) {
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < V::Q; ++q) acc += (double)f[s][q];
        rb[s] = acc;
        rho += acc;
      }
#pragma unroll
      for (int q = 1; q < V::Q; ++q) {
        R g = f[0][q];
#pragma unroll
        for (int s = 1; s < NC; ++s) g += f[s][q];
        if (V::cx(q)) jr[0] += (R)V::cx(q) * g;
        if (V::cy(q)) jr[1] += (R)V::cy(q) * g;
        if (V::cz(q)) jr[2] += (R)V::cz(q) * g;
      }
    }
    const double j[3] = {(double)jr[0], (double)jr[1], (double)jr[2]};
    double F[3];
    const double ps = psi[cell];
    force_at<LAT>(P, ps, [&](int a) { return psi[c.at(V::cx(a), V::cy(a), V::cz(a))]; }, F);
    double Ft[3], u[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      Ft[d] = F[d] + rho * P.accel[d];
      u[d] = (j[d] + 0.5 * Ft[d]) / rho;
    }
    if (rho_out)
#pragma unroll
      for (int s = 0; s < NC; ++s) rho_out[(size_t)s * P.cells + cell] = rb[s];
    if (u_out)
#pragma unroll
      for (int d = 0; d < D; ++d) u_out[(size_t)d * P.cells + cell] = u[d];
    if (p_out) {
      double Bn;
      p_out[cell] = eos_pressure<NC>(P, rb, &Bn);
    }
    if (psi_out) psi_out[cell] = ps;
#pragma unroll
    for (int s = 0; s < NC; ++s) vals[s] = rb[s];
#pragma unroll
    for (int d = 0; d < D; ++d) {
      vals[NC + d] = j[d] + 0.5 * Ft[d];
      vals[NC + D + d] = F[d];
    }
#pragma unroll
    for (int s = 0; s < NC; ++s) vals[NC + 2 * D + s] = rb[s] < 0.0 ? 1.0 : 0.0;
  }
  block_partials<K>(vals, partials);
}

// canonical post-streaming populations float64 [nc][Q][cells]
template <int LAT, int NC, int ST>
__global__ __launch_bounds__(kBlock) void k_export(KParams P, Pops<ST> in, double* __restrict__ f) {
  using V = VS<LAT>;
  using R = typename Pops<ST>::R;
  unsigned cell;
  if (!launch_cell(P, 0, P.nplanes, &cell)) return;
  const Coord c = make_coord(cell, P);
  const unsigned bits = P.bb ? P.bb[cell] : 0u;
#pragma unroll 1
  for (int s = 0; s < NC; ++s) {
    const auto cv = in.comp(s, V::Q, P.cells);
#pragma unroll
    for (int a = 0; a < V::Q; ++a) {
      const unsigned nbr = c.at(-V::cx(a), -V::cy(a), -V::cz(a));
      double v;
      if (!P.bb) v = (double)cv.get(a, nbr, (R)V::w(a));
      else if (bits >> kSolidBit) v = 0.0;   // solid cells hold no fluid
      else v = (double)pull_bb<LAT>(cv, a, bits, cell, nbr, (R)V::w(a));
      f[(size_t)(s * V::Q + a) * P.cells + cell] = v;
    }
  }
}

// mode 0: import canonical f (float64 [nc][Q][cells]);  mode 1: equilibrium of
// rho0 [nc][cells] and u0 [D][cells] (u0 may be NULL).  The base of the offset
// formats is the sum of the Q values stored at the cell.  With walls the stored
// direction a of a fluid cell y whose target y + e_a is solid is the population
// that bounces back into y as the opposite direction (bit opp(a) of y's mask),
// and solid cells store zeros.
template <int LAT, int NC, int ST>
__global__ __launch_bounds__(kBlock) void k_import(KParams P, Pops<ST> out, const double* __restrict__ f,
                                                  const double* __restrict__ rho0, const double* __restrict__ u0,
                                                  int mode) {
  using V = VS<LAT>;
  using R = typename Pops<ST>::R;
  constexpr int Q = V::Q;
  unsigned cell;
  if (!launch_cell(P, 0, P.nplanes, &cell)) return;
  const Coord c = make_coord(cell, P);
  const unsigned bits = P.bb ? P.bb[cell] : 0u;
  const bool solid = (bits >> kSolidBit) != 0u;
#pragma unroll 1
  for (int s = 0; s < NC; ++s) {
    double v[Q];
    double sum = 0.0;
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      const bool back = (bits >> V::opp(a)) & 1u;   // y + e_a solid: returns into y
      const unsigned dst = back ? cell : c.at(V::cx(a), V::cy(a), V::cz(a));
      const int ad = back ? V::opp(a) : a;          // canonical direction it becomes
      if (solid) {
        v[a] = 0.0;
      } else if (mode == 0) {
        v[a] = f[(size_t)(s * Q + ad) * P.cells + dst];
      } else {
        const double r = rho0[(size_t)s * P.cells + dst];
        double ux = 0.0, uy = 0.0, uz = 0.0;
        if (u0) {
          ux = u0[dst];
          uy = u0[(size_t)P.cells + dst];
          if (V::D == 3) uz = u0[(size_t)2 * P.cells + dst];
        }
        v[a] = feq<LAT, double>(ad, r, ux, uy, uz, ux * ux + uy * uy + uz * uz);
      }
      sum += v[a];
    }
    R vr[Q];
#pragma unroll
    for (int a = 0; a < Q; ++a) vr[a] = (R)v[a];
    out.comp(s, Q, P.cells).template put_all<Q>(cell, vr, sum, [](int a) { return (R)V::w(a); });
  }
}

}  // namespace lbmk
