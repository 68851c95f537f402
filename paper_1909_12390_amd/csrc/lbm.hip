// Kernels and C ABI of the multi-component pseudo-potential LB step on gfx950.
//
// Two-pass schedule of one step (Sec. 3.4 order):
//   k_psi     : pull + decode the populations, cell-volume densities (float64),
//               mixture EOS and psi (Eqs. MCPengRobinson, psicorrected) -> psi[cells]
//   k_collide : pull + decode again, psi stencil (Eq. coupledMCforce), split
//               (Eq. distributionforce), velocity, collision with forcing
//               (Eq. LBE / equilibrium; exact-difference method), encode + store.
// The fused schedule (lbm_fused.hpp) does the same arithmetic in one launch.
// Pull streaming over ping-pong copies: the kernel at cell x reads direction a
// from cell x - e_a of the "in" copy and writes its post-collision populations at
// x of the "out" copy, so no cell is read and written by different threads.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "lbm.h"
#include "lbm_fused.hpp"
#include "lbm_internal.hpp"
#include "lbm_kernels.hpp"

namespace {
thread_local char g_err[512] = "";
}

lbm_status lbm_fail(lbm_status code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

extern "C" const char* lbm_last_error(void) { return g_err; }

namespace lbmk {

constexpr int kBlock = 256;
constexpr int kMaxRed = LBM_MAX_NC + 6;   // reduction width: nc masses + 2 * D

// ---------------------------------------------------------------------------
// pass 1: densities -> EOS -> psi
// ---------------------------------------------------------------------------
template <int LAT, int NC, int ST>
__global__ __launch_bounds__(kBlock) void k_psi(KParams P, Pops<ST> in, double* __restrict__ psi) {
  using V = VS<LAT>;
  const int cell = blockIdx.x * kBlock + threadIdx.x;
  if (cell >= P.cells) return;
  const Coord c = make_coord(cell, P);
  double rb[NC];
#pragma unroll
  for (int s = 0; s < NC; ++s) {
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < V::Q; ++a)
      acc += (double)in.get(s, a, V::Q, c.at(-V::cx(a), -V::cy(a), -V::cz(a), P.nx, P.ny), P.cells,
                            (typename Pops<ST>::R)V::w(a));
    rb[s] = acc;
  }
  psi[cell] = eos_psi<NC>(P, rb);
}

// total force of Eq. (coupledMCforce) at one cell from psi(x) and its neighbours
template <int LAT, typename PsiAt>
__device__ __forceinline__ void force_at(const KParams& P, double ps, PsiAt psi_at, double* F) {
  using V = VS<LAT>;
  double fx = 0.0, fy = 0.0, fz = 0.0;
  const double hb = 0.5 * (1.0 - P.beta);
#pragma unroll
  for (int a = 1; a < V::Q; ++a) {
    const double pn = psi_at(a);
    const double t = V::w(a) * pn * (P.beta * ps + hb * pn);
    if (V::cx(a)) fx += V::cx(a) * t;
    if (V::cy(a)) fy += V::cy(a) * t;
    if (V::cz(a)) fz += V::cz(a) * t;
  }
  F[0] = -P.G * fx;
  F[1] = -P.G * fy;
  F[2] = -P.G * fz;
}

// ---------------------------------------------------------------------------
// pass 2: force, split, collide, store
// ---------------------------------------------------------------------------
template <int LAT, int NC, int ST>
__global__ __launch_bounds__(kBlock) void k_collide(KParams P, Pops<ST> in, Pops<ST> out,
                                                   const double* __restrict__ psi) {
  using V = VS<LAT>;
  using R = typename Pops<ST>::R;
  constexpr int Q = V::Q;
  const int cell = blockIdx.x * kBlock + threadIdx.x;
  if (cell >= P.cells) return;
  const Coord c = make_coord(cell, P);
  R f[NC][Q];
  double rb[NC], j[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int s = 0; s < NC; ++s) {
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      const R v = in.get(s, a, Q, c.at(-V::cx(a), -V::cy(a), -V::cz(a), P.nx, P.ny), P.cells, (R)V::w(a));
      f[s][a] = v;
      acc += (double)v;
      if (V::cx(a)) j[0] += V::cx(a) * (double)v;
      if (V::cy(a)) j[1] += V::cy(a) * (double)v;
      if (V::cz(a)) j[2] += V::cz(a) * (double)v;
    }
    rb[s] = acc;
  }
  double F[3];
  force_at<LAT>(P, psi[cell], [&](int a) { return psi[c.at(V::cx(a), V::cy(a), V::cz(a), P.nx, P.ny)]; }, F);
  double u[3], Fs[NC][3], du[NC][3];
  cell_forces<NC>(P, rb, j, F, u, Fs, du);
#pragma unroll
  for (int s = 0; s < NC; ++s) collide_store<LAT, ST>(P, out, s, cell, f[s], rb[s], u, Fs[s], du[s]);
}

// ---------------------------------------------------------------------------
// macroscopic fields + per-block partial sums for the conservation totals
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <int K>
__device__ __forceinline__ void block_partials(double* vals, double* partials) {
  __shared__ double red[kBlock / 64][K];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const double s = wave_sum(vals[k]);
    if (lane == 0) red[wv][k] = s;
  }
  __syncthreads();
  if (threadIdx.x < K) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) s += red[w][threadIdx.x];
    partials[(size_t)blockIdx.x * K + threadIdx.x] = s;
  }
}

template <int LAT, int NC, int ST>
__global__ __launch_bounds__(kBlock) void k_moments(KParams P, Pops<ST> in, const double* __restrict__ psi,
                                                   double* rho_out, double* u_out, double* p_out, double* psi_out,
                                                   double* partials) {
  using V = VS<LAT>;
  using R = typename Pops<ST>::R;
  constexpr int Q = V::Q, D = V::D, K = NC + 2 * D;
  const int cell = blockIdx.x * kBlock + threadIdx.x;
  double vals[K];
#pragma unroll
  for (int k = 0; k < K; ++k) vals[k] = 0.0;
  if (cell < P.cells) {
    const Coord c = make_coord(cell, P);
    double rb[NC], j[3] = {0.0, 0.0, 0.0}, rho = 0.0;
#pragma unroll
    for (int s = 0; s < NC; ++s) {
      double acc = 0.0;
#pragma unroll
      for (int a = 0; a < Q; ++a) {
        const double v = (double)in.get(s, a, Q, c.at(-V::cx(a), -V::cy(a), -V::cz(a), P.nx, P.ny), P.cells, (R)V::w(a));
        acc += v;
        if (V::cx(a)) j[0] += V::cx(a) * v;
        if (V::cy(a)) j[1] += V::cy(a) * v;
        if (V::cz(a)) j[2] += V::cz(a) * v;
      }
      rb[s] = acc;
      rho += acc;
    }
    double F[3];
    const double ps = psi[cell];
    force_at<LAT>(P, ps, [&](int a) { return psi[c.at(V::cx(a), V::cy(a), V::cz(a), P.nx, P.ny)]; }, F);
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
  }
  block_partials<K>(vals, partials);
}

// sum of the per-block partials in a fixed order (one block)
__global__ __launch_bounds__(kBlock) void k_finish(const double* __restrict__ partials, int nblocks, int K,
                                                  double* totals) {
  __shared__ double red[kBlock];
  for (int k = 0; k < K; ++k) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += kBlock) s += partials[(size_t)b * K + k];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
      if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) totals[k] = red[0];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// state import / export / initialisation (pull layout: the stored direction a at
// cell y is the population that arrives at y + e_a)
// ---------------------------------------------------------------------------
template <int LAT, int NC, int ST>
__global__ __launch_bounds__(kBlock) void k_export(KParams P, Pops<ST> in, double* __restrict__ f) {
  using V = VS<LAT>;
  using R = typename Pops<ST>::R;
  const int cell = blockIdx.x * kBlock + threadIdx.x;
  if (cell >= P.cells) return;
  const Coord c = make_coord(cell, P);
#pragma unroll
  for (int s = 0; s < NC; ++s)
#pragma unroll
    for (int a = 0; a < V::Q; ++a)
      f[(size_t)(s * V::Q + a) * P.cells + cell] =
          (double)in.get(s, a, V::Q, c.at(-V::cx(a), -V::cy(a), -V::cz(a), P.nx, P.ny), P.cells, (R)V::w(a));
}

// mode 0: import canonical f (float64 [nc][Q][cells]);  mode 1: equilibrium of
// rho0 [nc][cells] and u0 [D][cells] (u0 may be NULL)
template <int LAT, int NC, int ST>
__global__ __launch_bounds__(kBlock) void k_import(KParams P, Pops<ST> out, const double* __restrict__ f,
                                                  const double* __restrict__ rho0, const double* __restrict__ u0,
                                                  int mode) {
  using V = VS<LAT>;
  using R = typename Pops<ST>::R;
  constexpr int Q = V::Q;
  const int cell = blockIdx.x * kBlock + threadIdx.x;
  if (cell >= P.cells) return;
  const Coord c = make_coord(cell, P);
#pragma unroll
  for (int s = 0; s < NC; ++s) {
    double v[Q];
    double sum = 0.0;
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      const int dst = c.at(V::cx(a), V::cy(a), V::cz(a), P.nx, P.ny);
      if (mode == 0) {
        v[a] = f[(size_t)(s * Q + a) * P.cells + dst];
      } else {
        const double r = rho0[(size_t)s * P.cells + dst];
        double ux = 0.0, uy = 0.0, uz = 0.0;
        if (u0) {
          ux = u0[dst];
          uy = u0[(size_t)P.cells + dst];
          if (V::D == 3) uz = u0[(size_t)2 * P.cells + dst];
        }
        v[a] = feq<LAT, double>(a, r, ux, uy, uz, ux * ux + uy * uy + uz * uz);
      }
      sum += v[a];
    }
    const R base = (R)sum;
    out.put_base(s, cell, P.cells, base);
#pragma unroll
    for (int a = 0; a < Q; ++a) out.put(s, a, Q, cell, P.cells, (R)v[a], base, (R)V::w(a));
  }
}

// ---------------------------------------------------------------------------
// dispatch table over (lattice, nc, storage)
// ---------------------------------------------------------------------------
struct Bufs {
  void* p0;   // F64: f;  offset: base
  void* p1;   // offset: r
};

template <int ST>
Pops<ST> make_pops(const Bufs& b);
template <>
Pops<LBM_F64> make_pops<LBM_F64>(const Bufs& b) {
  Pops<LBM_F64> p;
  p.f = (double*)b.p0;
  return p;
}
template <>
Pops<LBM_F32_OFS> make_pops<LBM_F32_OFS>(const Bufs& b) {
  Pops<LBM_F32_OFS> p;
  p.base = (float*)b.p0;
  p.r = (float*)b.p1;
  return p;
}
template <>
Pops<LBM_F16_OFS> make_pops<LBM_F16_OFS>(const Bufs& b) {
  Pops<LBM_F16_OFS> p;
  p.base = (float*)b.p0;
  p.r = (__half*)b.p1;
  return p;
}

struct Ops {
  void (*step_two_pass)(const KParams&, const Bufs&, const Bufs&, double*, hipStream_t);
  void (*step_fused)(const KParams&, const Bufs&, const Bufs&, const FusedShape&, hipStream_t);
  void (*moments)(const KParams&, const Bufs&, double*, double*, double*, double*, double*, double*, hipStream_t);
  void (*exp)(const KParams&, const Bufs&, double*, hipStream_t);
  void (*imp)(const KParams&, const Bufs&, const double*, const double*, const double*, int, hipStream_t);
};

inline int nblocks(int cells) { return (cells + kBlock - 1) / kBlock; }

template <int LAT, int NC, int ST>
struct OpsImpl {
  static void step_two_pass(const KParams& P, const Bufs& in, const Bufs& out, double* psi, hipStream_t st) {
    const int nb = nblocks(P.cells);
    hipLaunchKernelGGL((k_psi<LAT, NC, ST>), dim3(nb), dim3(kBlock), 0, st, P, make_pops<ST>(in), psi);
    hipLaunchKernelGGL((k_collide<LAT, NC, ST>), dim3(nb), dim3(kBlock), 0, st, P, make_pops<ST>(in),
                       make_pops<ST>(out), (const double*)psi);
  }
  static void step_fused(const KParams& P, const Bufs& in, const Bufs& out, const FusedShape& fs, hipStream_t st) {
    launch_fused<LAT, NC, ST>(P, make_pops<ST>(in), make_pops<ST>(out), fs, st);
  }
  static void moments(const KParams& P, const Bufs& in, double* psi, double* rho, double* u, double* p,
                      double* psi_out, double* partials, hipStream_t st) {
    const int nb = nblocks(P.cells);
    hipLaunchKernelGGL((k_psi<LAT, NC, ST>), dim3(nb), dim3(kBlock), 0, st, P, make_pops<ST>(in), psi);
    hipLaunchKernelGGL((k_moments<LAT, NC, ST>), dim3(nb), dim3(kBlock), 0, st, P, make_pops<ST>(in),
                       (const double*)psi, rho, u, p, psi_out, partials);
  }
  static void exp(const KParams& P, const Bufs& in, double* f, hipStream_t st) {
    hipLaunchKernelGGL((k_export<LAT, NC, ST>), dim3(nblocks(P.cells)), dim3(kBlock), 0, st, P,
                       make_pops<ST>(in), f);
  }
  static void imp(const KParams& P, const Bufs& out, const double* f, const double* rho0, const double* u0, int mode,
                  hipStream_t st) {
    hipLaunchKernelGGL((k_import<LAT, NC, ST>), dim3(nblocks(P.cells)), dim3(kBlock), 0, st, P,
                       make_pops<ST>(out), f, rho0, u0, mode);
  }
  static Ops ops() { return Ops{&step_two_pass, &step_fused, &moments, &exp, &imp}; }
};

template <int LAT, int NC>
Ops ops_for_storage(int st) {
  switch (st) {
    case LBM_F64: return OpsImpl<LAT, NC, LBM_F64>::ops();
    case LBM_F32_OFS: return OpsImpl<LAT, NC, LBM_F32_OFS>::ops();
    default: return OpsImpl<LAT, NC, LBM_F16_OFS>::ops();
  }
}

template <int LAT>
Ops ops_for_nc(int nc, int st) {
  switch (nc) {
    case 1: return ops_for_storage<LAT, 1>(st);
    case 2: return ops_for_storage<LAT, 2>(st);
    case 3: return ops_for_storage<LAT, 3>(st);
    default: return ops_for_storage<LAT, 4>(st);
  }
}

Ops ops_for(int lat, int nc, int st) {
  return lat == LBM_D2Q9 ? ops_for_nc<LBM_D2Q9>(nc, st) : ops_for_nc<LBM_D3Q19>(nc, st);
}

}  // namespace lbmk

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
using namespace lbmk;

struct lbm_ctx {
  lbm_mixture mix;
  lbm_params prm;
  KParams kp;
  Ops ops;
  FusedShape fshape;
  int Q, D, K;
  size_t cells;
  hipStream_t stream;
  Bufs pops[2];
  double* psi;
  double* partials;
  double* totals;
  int* err;
  int cur;
};

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  size_t pop0[2], pop1[2], psi, partials, totals, err, total;
};

bool make_layout(const lbm_params* prm, int nc, Layout* L) {
  const int Q = prm->lattice == LBM_D2Q9 ? 9 : 19;
  const size_t cells = (size_t)prm->nx * prm->ny * prm->nz;
  size_t off = 0;
  const size_t s = prm->storage == LBM_F64 ? 8 : (prm->storage == LBM_F32_OFS ? 4 : 2);
  for (int k = 0; k < 2; ++k) {
    if (prm->storage == LBM_F64) {
      L->pop0[k] = off;
      off = align_up(off + (size_t)nc * Q * cells * 8);
      L->pop1[k] = 0;
    } else {
      L->pop0[k] = off;
      off = align_up(off + (size_t)nc * cells * 4);
      L->pop1[k] = off;
      off = align_up(off + (size_t)nc * Q * cells * s);
    }
  }
  L->psi = off;
  off = align_up(off + cells * 8);
  L->partials = off;
  off = align_up(off + (size_t)nblocks((int)cells) * kMaxRed * 8);
  L->totals = off;
  off = align_up(off + 16 * 8);
  L->err = off;
  off = align_up(off + 64);
  L->total = off;
  return true;
}

lbm_status validate(const lbm_mixture* mix, const lbm_params* prm) {
  if (!mix || !prm) return lbm_fail(LBM_ERR_ARG, "mixture or params is NULL");
  if (mix->nc < 1 || mix->nc > LBM_MAX_NC) return lbm_fail(LBM_ERR_ARG, "nc must be in 1..4");
  if (prm->lattice != LBM_D2Q9 && prm->lattice != LBM_D3Q19) return lbm_fail(LBM_ERR_ARG, "unknown lattice");
  if (prm->collision != LBM_BGK && prm->collision != LBM_MRT) return lbm_fail(LBM_ERR_ARG, "unknown collision");
  if (prm->forcing != LBM_GUO && prm->forcing != LBM_EDM) return lbm_fail(LBM_ERR_ARG, "unknown forcing");
  if (prm->storage < LBM_F64 || prm->storage > LBM_F16_OFS) return lbm_fail(LBM_ERR_ARG, "unknown storage");
  if (prm->schedule != LBM_SCHED_TWO_PASS && prm->schedule != LBM_SCHED_FUSED)
    return lbm_fail(LBM_ERR_ARG, "unknown schedule");
  if (prm->schedule == LBM_SCHED_FUSED && !fused_supported(prm->lattice))
    return lbm_fail(LBM_ERR_UNSUPPORTED, "fused schedule not built for this lattice");
  if (prm->nx < 1 || prm->ny < 1 || prm->nz < 1) return lbm_fail(LBM_ERR_ARG, "box sides must be >= 1");
  if (prm->lattice == LBM_D2Q9 && prm->nz != 1) return lbm_fail(LBM_ERR_ARG, "D2Q9 needs nz == 1");
  const double cells = (double)prm->nx * prm->ny * prm->nz;
  const int Q = prm->lattice == LBM_D2Q9 ? 9 : 19;
  if (cells * mix->nc * Q >= 2147483647.0) return lbm_fail(LBM_ERR_ARG, "box too large for 32-bit plane indexing");
  if (!(prm->tau > 0.5)) return lbm_fail(LBM_ERR_ARG, "tau must exceed 0.5");
  if (!(prm->G < 0.0)) return lbm_fail(LBM_ERR_ARG, "G must be negative");
  if (!(prm->T > 0.0)) return lbm_fail(LBM_ERR_ARG, "T must be positive");
  if (!std::isfinite(prm->beta)) return lbm_fail(LBM_ERR_ARG, "beta must be finite");
  for (int i = 0; i < mix->nc; ++i) {
    if (!(prm->gamma[i] > 0.0 && prm->gamma[i] <= 1.0)) return lbm_fail(LBM_ERR_ARG, "gamma_%d outside (0, 1]", i);
    if (!(mix->a[i] > 0.0 && mix->b[i] > 0.0 && mix->M[i] > 0.0))
      return lbm_fail(LBM_ERR_ARG, "a, b, M must be positive");
    for (int j = 0; j < mix->nc; ++j)
      if (mix->k[i][j] != mix->k[j][i]) return lbm_fail(LBM_ERR_ARG, "k must be symmetric");
  }
  if (prm->collision == LBM_MRT)
    for (int k = 0; k < Q; ++k)
      if (!(prm->mrt_s[k] >= 0.0 && prm->mrt_s[k] < 2.0)) return lbm_fail(LBM_ERR_ARG, "MRT rate %d outside [0, 2)", k);
  if (!(mix->R > 0.0)) return lbm_fail(LBM_ERR_ARG, "R must be positive");
  return LBM_OK;
}

template <int LAT>
void fill_mrt(const lbm_params* prm, KParams* kp) {
  for (int k = 0; k < VS<LAT>::Q; ++k) kp->s_over_n[k] = prm->mrt_s[k] / mrow_norm2<LAT>(k);
}

lbm_status hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) return lbm_fail(LBM_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
  return LBM_OK;
}

}  // namespace

extern "C" lbm_status lbm_workspace_bytes(const lbm_mixture* mix, const lbm_params* prm, size_t* bytes) {
  lbm_status st = validate(mix, prm);
  if (st != LBM_OK) return st;
  if (!bytes) return lbm_fail(LBM_ERR_ARG, "bytes is NULL");
  Layout L;
  make_layout(prm, mix->nc, &L);
  *bytes = L.total;
  return LBM_OK;
}

extern "C" lbm_status lbm_init(const lbm_mixture* mix, const lbm_params* prm, void* ws, size_t ws_bytes,
                               const double* rho0, const double* u0, void* stream, lbm_ctx** out) {
  if (!out) return lbm_fail(LBM_ERR_ARG, "out is NULL");
  *out = nullptr;
  lbm_status st = validate(mix, prm);
  if (st != LBM_OK) return st;
  if (!ws || ((uintptr_t)ws % kAlign) != 0) return lbm_fail(LBM_ERR_ARG, "workspace must be 256-byte aligned");
  if (!rho0) return lbm_fail(LBM_ERR_ARG, "rho_bar0 is NULL");
  Layout L;
  make_layout(prm, mix->nc, &L);
  if (ws_bytes < L.total) return lbm_fail(LBM_ERR_ARG, "workspace too small: %zu < %zu", ws_bytes, L.total);

  lbm_ctx* c = new (std::nothrow) lbm_ctx();
  if (!c) return lbm_fail(LBM_ERR_ARG, "out of host memory");
  c->mix = *mix;
  c->prm = *prm;
  c->Q = prm->lattice == LBM_D2Q9 ? 9 : 19;
  c->D = prm->lattice == LBM_D2Q9 ? 2 : 3;
  c->K = mix->nc + 2 * c->D;
  c->cells = (size_t)prm->nx * prm->ny * prm->nz;
  c->stream = (hipStream_t)stream;
  char* base = (char*)ws;
  for (int k = 0; k < 2; ++k) {
    c->pops[k].p0 = base + L.pop0[k];
    c->pops[k].p1 = prm->storage == LBM_F64 ? nullptr : base + L.pop1[k];
  }
  c->psi = (double*)(base + L.psi);
  c->partials = (double*)(base + L.partials);
  c->totals = (double*)(base + L.totals);
  c->err = (int*)(base + L.err);
  c->cur = 0;

  KParams& kp = c->kp;
  std::memset(&kp, 0, sizeof(kp));
  kp.nx = prm->nx;
  kp.ny = prm->ny;
  kp.nz = prm->nz;
  kp.cells = (int)c->cells;
  kp.collision = prm->collision;
  kp.forcing = prm->forcing;
  kp.RT = mix->R * prm->T;
  kp.G = prm->G;
  kp.beta = prm->beta;
  kp.omega = 1.0 / prm->tau;
  double aa[LBM_MAX_NC];
  lbm_internal_aalpha(mix, prm->T, aa);
  for (int i = 0; i < mix->nc; ++i) {
    kp.b[i] = mix->b[i];
    kp.invM[i] = 1.0 / mix->M[i];
    kp.gamma[i] = prm->gamma[i];
    for (int j = 0; j < mix->nc; ++j) kp.aa[i][j] = std::sqrt(aa[i] * aa[j]) * (1.0 - mix->k[i][j]);
  }
  if (prm->collision == LBM_MRT) {
    if (prm->lattice == LBM_D2Q9) fill_mrt<LBM_D2Q9>(prm, &kp);
    else fill_mrt<LBM_D3Q19>(prm, &kp);
  }
  for (int d = 0; d < 3; ++d) kp.accel[d] = (d < c->D) ? prm->accel[d] : 0.0;
  kp.err = c->err;
  c->ops = ops_for(prm->lattice, mix->nc, prm->storage);
  c->fshape = fused_shape(prm->lattice, prm->nx, prm->ny, prm->nz);

  st = hip_check(hipMemsetAsync(c->err, 0, sizeof(int), c->stream), "hipMemsetAsync(err)");
  if (st != LBM_OK) {
    delete c;
    return st;
  }
  c->ops.imp(kp, c->pops[0], nullptr, rho0, u0, 1, c->stream);
  st = hip_check(hipGetLastError(), "init launch");
  if (st != LBM_OK) {
    delete c;
    return st;
  }
  *out = c;
  return LBM_OK;
}

extern "C" lbm_status lbm_step(lbm_ctx* c, int nsteps) {
  if (!c || nsteps < 0) return lbm_fail(LBM_ERR_ARG, "bad lbm_step arguments");
  for (int i = 0; i < nsteps; ++i) {
    const Bufs& in = c->pops[c->cur];
    const Bufs& out = c->pops[1 - c->cur];
    if (c->prm.schedule == LBM_SCHED_FUSED) c->ops.step_fused(c->kp, in, out, c->fshape, c->stream);
    else c->ops.step_two_pass(c->kp, in, out, c->psi, c->stream);
    c->cur = 1 - c->cur;
  }
  return hip_check(hipGetLastError(), "step launch");
}

extern "C" lbm_status lbm_check(lbm_ctx* c) {
  if (!c) return lbm_fail(LBM_ERR_ARG, "ctx is NULL");
  lbm_status st = hip_check(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  if (st != LBM_OK) return st;
  int flag = 0;
  st = hip_check(hipMemcpy(&flag, c->err, sizeof(int), hipMemcpyDeviceToHost), "hipMemcpy(err)");
  if (st != LBM_OK) return st;
  if (flag) return lbm_fail(LBM_ERR_DOMAIN, "EOS/psi domain violation or non-finite value on the device");
  return LBM_OK;
}

extern "C" lbm_status lbm_clear_error(lbm_ctx* c) {
  if (!c) return lbm_fail(LBM_ERR_ARG, "ctx is NULL");
  return hip_check(hipMemsetAsync(c->err, 0, sizeof(int), c->stream), "hipMemsetAsync(err)");
}

extern "C" lbm_status lbm_moments(lbm_ctx* c, double* rho, double* u, double* p, double* psi, double* totals) {
  if (!c) return lbm_fail(LBM_ERR_ARG, "ctx is NULL");
  c->ops.moments(c->kp, c->pops[c->cur], c->psi, rho, u, p, psi, c->partials, c->stream);
  lbm_status st = hip_check(hipGetLastError(), "moments launch");
  if (st != LBM_OK) return st;
  if (totals) {
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kBlock), 0, c->stream, (const double*)c->partials,
                       nblocks((int)c->cells), c->K, c->totals);
    st = hip_check(hipGetLastError(), "finish launch");
    if (st != LBM_OK) return st;
    st = hip_check(hipMemcpyAsync(totals, c->totals, sizeof(double) * c->K, hipMemcpyDeviceToHost, c->stream),
                   "hipMemcpyAsync(totals)");
    if (st != LBM_OK) return st;
    return lbm_check(c);
  }
  return LBM_OK;
}

extern "C" lbm_status lbm_get_populations(lbm_ctx* c, double* f) {
  if (!c || !f) return lbm_fail(LBM_ERR_ARG, "bad lbm_get_populations arguments");
  c->ops.exp(c->kp, c->pops[c->cur], f, c->stream);
  return hip_check(hipGetLastError(), "export launch");
}

extern "C" lbm_status lbm_set_populations(lbm_ctx* c, const double* f) {
  if (!c || !f) return lbm_fail(LBM_ERR_ARG, "bad lbm_set_populations arguments");
  c->ops.imp(c->kp, c->pops[c->cur], f, nullptr, nullptr, 0, c->stream);
  return hip_check(hipGetLastError(), "import launch");
}

extern "C" void lbm_destroy(lbm_ctx* c) { delete c; }
