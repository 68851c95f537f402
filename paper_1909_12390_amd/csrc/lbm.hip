// C ABI of the multi-component pseudo-potential LB step on gfx950 (host side).
//
// One step (Sec. 3.4 order) is two kernel passes (lbm_kernels.hpp):
//   k_psi     : pull + decode the populations, cell-volume densities (float64),
//               mixture EOS and psi (Eqs. MCPengRobinson, psicorrected) -> psi[cells]
//   k_collide : pull + decode again, psi stencil (Eq. coupledMCforce), split
//               (Eq. distributionforce), velocity, collision with forcing
//               (Eq. LBE / equilibrium; exact-difference method), encode + store.
// Pull streaming over ping-pong copies: the kernel at cell x reads direction a
// from cell x - e_a of the "in" copy and writes its post-collision populations at
// x of the "out" copy, so no cell is read and written by different threads.
// The blocked schedule runs both passes slab by slab along the slowest axis.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "lbm.h"
#include "lbm_ctx.hpp"
#include "lbm_walls.hpp"
#include "lbm_internal.hpp"

namespace {
thread_local char g_err[512] = "";
}

// Scratch of lbm_moments_noalloc: the per-block partial sums of the conservation
// totals and the finished totals, in a file-scope device array instead of the
// context's workspace.  Every GPU the library runs on holds its own copy until the
// process ends.  Host code never uses the array's name as an address: lbm_init
// looks up its device address once per device (hipGetSymbolAddress, with that
// device current) and lbm_moments_noalloc uses only that address.
constexpr size_t kNoallocScratchBytes = size_t(1) << 20;
constexpr size_t kNoallocTotalsBytes = 256;   // totals (<= kMaxRed doubles) at the end of the array
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];
static_assert(lbmk::kMaxRed * sizeof(double) <= kNoallocTotalsBytes, "totals do not fit the scratch's tail");

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];   // device address of `scratch` per device, null until looked up
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

// sum of the per-block partials (total-major [K][nblocks], see block_partials) in a
// fixed order, one block: thread t adds blocks t, t + kBlock, ... of every total in
// turn (coalesced across the threads, eight blocks' values loaded before they are
// added in that same order), then a fixed tree over the threads, all K at once
__global__ __launch_bounds__(kBlock) void k_finish(const double* __restrict__ partials, int nblocks, int K,
                                                  double* totals) {
  __shared__ double red[kMaxRed][kBlock];
  double s[kMaxRed];
#pragma unroll
  for (int k = 0; k < kMaxRed; ++k) s[k] = 0.0;
  constexpr int U = 8;
  int b = threadIdx.x;
  for (; b + (U - 1) * kBlock < nblocks; b += U * kBlock) {
    double v[U][kMaxRed];
#pragma unroll
    for (int k = 0; k < kMaxRed; ++k)
#pragma unroll
      for (int u = 0; u < U; ++u) v[u][k] = k < K ? partials[(size_t)k * nblocks + b + u * kBlock] : 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < kMaxRed; ++k) s[k] += v[u][k];
  }
  for (; b < nblocks; b += kBlock)
#pragma unroll
    for (int k = 0; k < kMaxRed; ++k)
      if (k < K) s[k] += partials[(size_t)k * nblocks + b];
#pragma unroll
  for (int k = 0; k < kMaxRed; ++k) red[k][threadIdx.x] = s[k];
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
#pragma unroll
      for (int k = 0; k < kMaxRed; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
    __syncthreads();
  }
  if ((int)threadIdx.x < K) totals[threadIdx.x] = red[threadIdx.x][0];
}

}  // namespace lbmk

using namespace lbmk;

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  size_t pop0[2], pop1[2], psi, partials, totals, err, total;
};

size_t storage_bytes(int storage) { return storage == LBM_F64 ? 8 : (storage == LBM_F32_OFS ? 4 : 2); }

void make_layout(const lbm_params* prm, int nc, Layout* L) {
  const int Q = prm->lattice == LBM_D2Q9 ? 9 : 19;
  const size_t cells = (size_t)prm->nx * prm->ny * prm->nz;
  const size_t s = storage_bytes(prm->storage);
  size_t off = 0;
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
  off = align_up(off + (size_t)nblocks_for((int)cells) * kMaxRed * 8);
  L->totals = off;
  off = align_up(off + 16 * 8);
  L->err = off;
  off = align_up(off + 64);
  L->total = off;
}

lbm_status validate(const lbm_mixture* mix, const lbm_params* prm) {
  if (!mix || !prm) return lbm_fail(LBM_ERR_ARG, "mixture or params is NULL");
  if (mix->nc < 1 || mix->nc > LBM_MAX_NC) return lbm_fail(LBM_ERR_ARG, "nc must be in 1..4");
  if (prm->lattice != LBM_D2Q9 && prm->lattice != LBM_D3Q19) return lbm_fail(LBM_ERR_ARG, "unknown lattice");
  if (prm->collision != LBM_BGK && prm->collision != LBM_MRT) return lbm_fail(LBM_ERR_ARG, "unknown collision");
  if (prm->forcing != LBM_GUO && prm->forcing != LBM_EDM) return lbm_fail(LBM_ERR_ARG, "unknown forcing");
  if (prm->storage < LBM_F64 || prm->storage > LBM_F16_OFS) return lbm_fail(LBM_ERR_ARG, "unknown storage");
  if (prm->schedule != LBM_SCHED_TWO_PASS && prm->schedule != LBM_SCHED_BLOCKED &&
      prm->schedule != LBM_SCHED_OVERLAP)
    return lbm_fail(LBM_ERR_ARG, "unknown schedule");
  if (prm->slab_planes < 0) return lbm_fail(LBM_ERR_ARG, "slab_planes must be >= 0");
  if (prm->nx < 1 || prm->ny < 1 || prm->nz < 1) return lbm_fail(LBM_ERR_ARG, "box sides must be >= 1");
  if (prm->lattice == LBM_D2Q9 && prm->nz != 1) return lbm_fail(LBM_ERR_ARG, "D2Q9 needs nz == 1");
  const double cells = (double)prm->nx * prm->ny * prm->nz;
  const double Qd = prm->lattice == LBM_D2Q9 ? 9.0 : 19.0;
  // population planes are addressed with 32-bit byte offsets: one component's planes
  // (float64), all components' interleaved planes (offset formats)
  const double sb = prm->storage == LBM_F64 ? 8.0 : (prm->storage == LBM_F32_OFS ? 4.0 : 2.0);
  const double span = prm->storage == LBM_F64 ? cells * 8.0 * Qd : cells * sb * Qd * mix->nc;
  if (span >= 4294967295.0)
    return lbm_fail(LBM_ERR_ARG, "box too large: the population planes addressed together must stay below 4 GiB");
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
  const int Q = prm->lattice == LBM_D2Q9 ? 9 : 19;
  if (prm->collision == LBM_MRT)
    for (int k = 0; k < Q; ++k)
      if (!(prm->mrt_s[k] >= 0.0 && prm->mrt_s[k] < 2.0)) return lbm_fail(LBM_ERR_ARG, "MRT rate %d outside [0, 2)", k);
  if (!(mix->R > 0.0)) return lbm_fail(LBM_ERR_ARG, "R must be positive");
  return LBM_OK;
}

template <int LAT>
void fill_mrt(const lbm_params* prm, KParams* kp) {
  kp->mrt_rows = 0;
  for (int k = 0; k < VS<LAT>::Q; ++k) {
    kp->mrt_c[k] = (1.0 - prm->mrt_s[k]) / mrow_norm2<LAT>(k);
    if (kp->mrt_c[k] != 0.0) kp->mrt_rows |= 1u << k;
  }
}

lbm_status hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) return lbm_fail(LBM_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
  return LBM_OK;
}

// Enqueue one step; mark(k) runs after every psi (k = 0) / collide (k = 1) launch.
// OVERLAP: psi slabs on the aux stream (in the order last, 0, 1, ...), each collide
// slab on the context's stream after the psi events of slabs k-1, k, k+1; the aux
// stream first waits for the previous step's work on the context's stream.
void enqueue_overlap(lbm_ctx* c, const Bufs& in, const Bufs& out) {
  const int np = c->kp.nplanes, sl = c->slab;
  const int ns = (np + sl - 1) / sl;
  hipEvent_t* done = c->ev;            // [ns] psi of slab k done
  hipEvent_t boundary = c->ev[ns];
  hipEventRecord(boundary, c->stream);
  hipStreamWaitEvent(c->aux, boundary, 0);
  for (int i = 0; i < ns; ++i) {
    const int k = (i == 0) ? ns - 1 : i - 1;
    const int p0 = k * sl, n = std::min(sl, np - p0);
    c->ops.psi(c->kp, in, c->sc, p0, n, c->aux);
    hipEventRecord(done[k], c->aux);
  }
  for (int k = 0; k < ns; ++k) {
    hipStreamWaitEvent(c->stream, done[(k + ns - 1) % ns], 0);
    hipStreamWaitEvent(c->stream, done[k], 0);
    hipStreamWaitEvent(c->stream, done[(k + 1) % ns], 0);
    const int p0 = k * sl, n = std::min(sl, np - p0);
    c->ops.collide(c->kp, in, out, c->sc, p0, n, c->stream);
  }
}

template <typename Mark>
void enqueue_step(lbm_ctx* c, Mark mark) {
  const Bufs& in = c->pops[c->cur];
  const Bufs& out = c->pops[1 - c->cur];
  const int np = c->kp.nplanes;
  if (c->prm.schedule == LBM_SCHED_OVERLAP && c->aux) {
    enqueue_overlap(c, in, out);
    mark(1);
  } else if (c->prm.schedule == LBM_SCHED_TWO_PASS || c->slab >= np) {
    c->ops.psi(c->kp, in, c->sc, 0, np, c->stream);
    mark(0);
    c->ops.collide(c->kp, in, out, c->sc, 0, np, c->stream);
    mark(1);
  } else {
    for (int m0 = 0; m0 < np; m0 += c->slab) {
      const int n = std::min(c->slab, np - m0);
      if (n + 2 >= np) c->ops.psi(c->kp, in, c->sc, 0, np, c->stream);
      else c->ops.psi(c->kp, in, c->sc, m0 == 0 ? np - 1 : m0 - 1, n + 2, c->stream);
      mark(0);
      c->ops.collide(c->kp, in, out, c->sc, m0, n, c->stream);
      mark(1);
    }
  }
  c->cur = 1 - c->cur;
}

int launches_per_step(const lbm_ctx* c) {
  const int np = c->kp.nplanes;
  if (c->prm.schedule == LBM_SCHED_OVERLAP && c->aux) return 1;
  if (c->prm.schedule == LBM_SCHED_TWO_PASS || c->slab >= np) return 2;
  return 2 * ((np + c->slab - 1) / c->slab);
}

// A copy of prm whose gamma, when given as all zero, is the two-phase flash's at
// (T, p_flash, z_flash): Eq. (gamma) on the phases of Sec. 3.2.
lbm_status resolve_gamma(const lbm_mixture* mix, const lbm_params* prm, lbm_params* out) {
  if (!mix || !prm) return lbm_fail(LBM_ERR_ARG, "mixture or params is NULL");
  if (mix->nc < 1 || mix->nc > LBM_MAX_NC) return lbm_fail(LBM_ERR_ARG, "nc must be in 1..4");
  *out = *prm;
  for (int i = 0; i < mix->nc; ++i)
    if (prm->gamma[i] != 0.0) return LBM_OK;
  lbm_flash_result fr;
  const lbm_status st = lbm_flash(mix, prm->T, prm->p_flash, prm->z_flash, &fr);
  if (st != LBM_OK) return st;
  for (int i = 0; i < mix->nc; ++i) out->gamma[i] = fr.gamma[i];
  return LBM_OK;
}

}  // namespace

extern "C" lbm_status lbm_workspace_bytes(const lbm_mixture* mix, const lbm_params* prm_in, size_t* bytes) {
  lbm_params resolved;
  lbm_status st = resolve_gamma(mix, prm_in, &resolved);
  if (st != LBM_OK) return st;
  const lbm_params* prm = &resolved;
  st = validate(mix, prm);
  if (st != LBM_OK) return st;
  if (!bytes) return lbm_fail(LBM_ERR_ARG, "bytes is NULL");
  Layout L;
  make_layout(prm, mix->nc, &L);
  *bytes = L.total;
  return LBM_OK;
}

namespace {
// The device address of `scratch` on `dev` (the current device), looked up once per
// device; later calls return the kept address.
lbm_status noalloc_scratch_address(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return lbm_fail(LBM_ERR_ARG, "device index %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev]) return LBM_OK;
  void* p = nullptr;
  lbm_status st = hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
  if (st != LBM_OK) return st;
  if (!p) return lbm_fail(LBM_ERR_HIP, "hipGetSymbolAddress(scratch) returned a null address");
  g_scratch_ptr[dev] = p;
  return LBM_OK;
}
}  // namespace

extern "C" lbm_status lbm_init(const lbm_mixture* mix, const lbm_params* prm_in, void* ws, size_t ws_bytes,
                               const double* rho0, const double* u0, void* stream, lbm_ctx** out) {
  if (!out) return lbm_fail(LBM_ERR_ARG, "out is NULL");
  *out = nullptr;
  lbm_params resolved;
  lbm_status st = resolve_gamma(mix, prm_in, &resolved);
  if (st != LBM_OK) return st;
  const lbm_params* prm = &resolved;
  st = validate(mix, prm);
  if (st != LBM_OK) return st;
  int dev = -1;
  st = hip_check(hipGetDevice(&dev), "hipGetDevice");
  if (st != LBM_OK) return st;
  st = noalloc_scratch_address(dev);
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
  c->K = 2 * mix->nc + 2 * c->D;
  c->cells = (size_t)prm->nx * prm->ny * prm->nz;
  c->stream = (hipStream_t)stream;
  char* base = (char*)ws;
  for (int k = 0; k < 2; ++k) {
    c->pops[k].p0 = base + L.pop0[k];
    c->pops[k].p1 = prm->storage == LBM_F64 ? nullptr : base + L.pop1[k];
    c->pops[k].nc = mix->nc;
  }
  c->psi = (double*)(base + L.psi);
  c->sc.psi = c->psi;
  c->partials = (double*)(base + L.partials);
  c->totals = (double*)(base + L.totals);
  c->err = (int*)(base + L.err);
  c->cur = 0;
  c->device = dev;

  KParams& kp = c->kp;
  std::memset(&kp, 0, sizeof(kp));
  kp.nx = prm->nx;
  kp.ny = prm->ny;
  kp.nz = prm->nz;
  kp.cells = (int)c->cells;
  kp.plane_cells = prm->lattice == LBM_D2Q9 ? prm->nx : prm->nx * prm->ny;
  kp.nplanes = prm->lattice == LBM_D2Q9 ? prm->ny : prm->nz;
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
  c->ops = prm->lattice == LBM_D2Q9 ? ops_d2q9(mix->nc, prm->storage, prm->collision, prm->forcing)
                                    : ops_d3q19(mix->nc, prm->storage, prm->collision, prm->forcing);
  c->adj = prm->lattice == LBM_D2Q9 ? adj_ops_d2q9(mix->nc, prm->storage, prm->collision, prm->forcing)
                                    : adj_ops_d3q19(mix->nc, prm->storage, prm->collision, prm->forcing);
  if (prm->slab_planes > 0) {
    c->slab = prm->slab_planes;
  } else if (prm->schedule == LBM_SCHED_OVERLAP) {
    c->slab = std::max(1, (kp.nplanes + 7) / 8);
  } else {
    // about 64 MiB of population input (+ base) per slab
    const double plane_bytes = (double)kp.plane_cells * mix->nc *
                               (c->Q * (double)storage_bytes(prm->storage) + (prm->storage == LBM_F64 ? 0.0 : 4.0));
    c->slab = std::max(1, (int)((64.0 * 1048576.0) / plane_bytes));
  }

  if (prm->schedule == LBM_SCHED_OVERLAP) {
    const int ns = (kp.nplanes + c->slab - 1) / c->slab;
    st = hip_check(hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking), "create overlap stream");
    if (st == LBM_OK) {
      c->ev = new (std::nothrow) hipEvent_t[ns + 1];
      if (!c->ev) st = lbm_fail(LBM_ERR_ARG, "out of host memory");
    }
    for (int k = 0; st == LBM_OK && k <= ns; ++k) {
      st = hip_check(hipEventCreateWithFlags(&c->ev[k], hipEventDisableTiming), "create overlap event");
      if (st == LBM_OK) c->nev = k + 1;
    }
    if (st != LBM_OK) {
      delete c;
      return st;
    }
  }
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
  int left = nsteps;
  if (c->graph_steps > 0 && c->prm.schedule != LBM_SCHED_OVERLAP) {
    while (left >= c->graph_steps) {
      const int p = c->cur;
      if (!c->graph[p]) {
        hipGraph_t g = nullptr;
        lbm_status st = hip_check(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal), "begin capture");
        if (st != LBM_OK) return st;
        for (int i = 0; i < c->graph_steps; ++i) enqueue_step(c, [](int) {});
        st = hip_check(hipStreamEndCapture(c->stream, &g), "end capture");
        c->cur = p;   // capture only recorded the launches; the replay below performs them
        if (st != LBM_OK) return st;
        st = hip_check(hipGraphInstantiate(&c->graph[p], g, nullptr, nullptr, 0), "instantiate graph");
        hipGraphDestroy(g);
        if (st != LBM_OK) return st;
      }
      lbm_status st = hip_check(hipGraphLaunch(c->graph[p], c->stream), "graph launch");
      if (st != LBM_OK) return st;
      left -= c->graph_steps;   // an even number of steps keeps the buffer parity
    }
  }
  for (int i = 0; i < left; ++i) enqueue_step(c, [](int) {});
  return hip_check(hipGetLastError(), "step launch");
}

extern "C" lbm_status lbm_set_graph_steps(lbm_ctx* c, int steps) {
  if (!c || steps < 0) return lbm_fail(LBM_ERR_ARG, "bad lbm_set_graph_steps arguments");
  if (steps > 0 && !c->stream) return lbm_fail(LBM_ERR_ARG, "graph capture needs a non-default stream");
  c->drop_graphs();
  c->graph_steps = steps > 0 ? (steps + 1) / 2 * 2 : 0;
  return LBM_OK;
}

extern "C" lbm_status lbm_step_timed(lbm_ctx* c, int nsteps, double* kernel_ms) {
  if (!c || nsteps < 0 || !kernel_ms) return lbm_fail(LBM_ERR_ARG, "bad lbm_step_timed arguments");
  kernel_ms[0] = kernel_ms[1] = 0.0;
  if (nsteps == 0) return LBM_OK;
  const int nev = nsteps * launches_per_step(c) + 1;
  hipEvent_t* ev = new (std::nothrow) hipEvent_t[nev];
  int* kind = new (std::nothrow) int[nev];
  if (!ev || !kind) {
    delete[] ev;
    delete[] kind;
    return lbm_fail(LBM_ERR_ARG, "out of host memory");
  }
  int made = 0;
  lbm_status st = LBM_OK;
  for (; made < nev; ++made) {
    st = hip_check(hipEventCreate(&ev[made]), "hipEventCreate");
    if (st != LBM_OK) break;
  }
  if (st == LBM_OK) {
    int e = 0;
    hipEventRecord(ev[e++], c->stream);
    for (int i = 0; i < nsteps; ++i)
      enqueue_step(c, [&](int k) {
        kind[e] = k;
        hipEventRecord(ev[e++], c->stream);
      });
    st = hip_check(hipGetLastError(), "step launch");
    if (st == LBM_OK) st = hip_check(hipEventSynchronize(ev[nev - 1]), "hipEventSynchronize");
    if (st == LBM_OK) {
      for (int k = 1; k < nev; ++k) {
        float ms = 0.0f;
        hipEventElapsedTime(&ms, ev[k - 1], ev[k]);
        kernel_ms[kind[k]] += ms;
      }
    }
  }
  for (int k = 0; k < made; ++k) hipEventDestroy(ev[k]);
  delete[] ev;
  delete[] kind;
  return st;
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

extern "C" lbm_status lbm_set_gamma(lbm_ctx* c, const double* gamma) {
  if (!c || !gamma) return lbm_fail(LBM_ERR_ARG, "bad lbm_set_gamma arguments");
  for (int i = 0; i < c->mix.nc; ++i)
    if (!(gamma[i] > 0.0 && gamma[i] <= 1.0)) return lbm_fail(LBM_ERR_ARG, "gamma_%d outside (0, 1]", i);
  for (int i = 0; i < c->mix.nc; ++i) {
    c->prm.gamma[i] = gamma[i];
    c->kp.gamma[i] = gamma[i];   // kernel arguments: the next launch uses the new values
  }
  c->drop_graphs();              // captured launches hold the old values
  return LBM_OK;
}

extern "C" lbm_status lbm_clear_error(lbm_ctx* c) {
  if (!c) return lbm_fail(LBM_ERR_ARG, "ctx is NULL");
  return hip_check(hipMemsetAsync(c->err, 0, sizeof(int), c->stream), "hipMemsetAsync(err)");
}

extern "C" lbm_status lbm_moments(lbm_ctx* c, double* rho, double* u, double* p, double* psi, double* totals) {
  if (!c) return lbm_fail(LBM_ERR_ARG, "ctx is NULL");
  c->ops.moments(c->kp, c->pops[c->cur], c->sc, rho, u, p, psi, c->partials, c->stream);
  lbm_status st = hip_check(hipGetLastError(), "moments launch");
  if (st != LBM_OK) return st;
  if (totals) {
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kBlock), 0, c->stream, (const double*)c->partials,
                       nblocks_for((int)c->cells), c->K, c->totals);
    st = hip_check(hipGetLastError(), "finish launch");
    if (st != LBM_OK) return st;
    st = hip_check(hipMemcpyAsync(totals, c->totals, sizeof(double) * c->K, hipMemcpyDeviceToHost, c->stream),
                   "hipMemcpyAsync(totals)");
    if (st != LBM_OK) return st;
    return lbm_check(c);
  }
  return LBM_OK;
}

extern "C" lbm_status lbm_moments_noalloc(lbm_ctx* c, double* rho, double* u, double* p, double* psi,
                                          double* totals) {
  if (!c) return lbm_fail(LBM_ERR_ARG, "ctx is NULL");
  const size_t nb = (size_t)nblocks_for((int)c->cells);
  const size_t need = nb * (size_t)c->K * sizeof(double);
  if (need > kNoallocScratchBytes - kNoallocTotalsBytes)
    return lbm_fail(LBM_ERR_ARG,
                    "box too large for lbm_moments_noalloc: its partial sums need %zu bytes, the static "
                    "scratch holds %zu (use lbm_moments)",
                    need, kNoallocScratchBytes - kNoallocTotalsBytes);
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    base = g_scratch_ptr[c->device];   // set by lbm_init on this device
  }
  if (!base) return lbm_fail(LBM_ERR_HIP, "no scratch address for device %d", c->device);
  double* partials = (double*)base;
  double* tot = (double*)((char*)base + kNoallocScratchBytes - kNoallocTotalsBytes);
  // k_moments writes every block's K partials and k_finish every total: nothing in
  // the scratch needs clearing (it keeps the last call's values)
  c->ops.moments(c->kp, c->pops[c->cur], c->sc, rho, u, p, psi, partials, c->stream);
  lbm_status st = hip_check(hipGetLastError(), "moments launch");
  if (st != LBM_OK) return st;
  if (totals) {
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kBlock), 0, c->stream, (const double*)partials, (int)nb, c->K, tot);
    st = hip_check(hipGetLastError(), "finish launch");
    if (st != LBM_OK) return st;
    st = hip_check(hipMemcpyAsync(totals, tot, sizeof(double) * c->K, hipMemcpyDeviceToHost, c->stream),
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

extern "C" lbm_status lbm_set_solid(lbm_ctx* c, const unsigned char* solid, double psi_wall) {
  if (!c) return lbm_fail(LBM_ERR_ARG, "ctx is NULL");
  if (solid && !(std::isfinite(psi_wall) && psi_wall >= 0.0))
    return lbm_fail(LBM_ERR_ARG, "psi_wall must be finite and >= 0");
  // canonical populations under the current walls, re-imported under the new ones
  const size_t fbytes = sizeof(double) * (size_t)c->mix.nc * c->Q * c->cells;
  double* tmp = nullptr;
  lbm_status st = hip_check(hipMalloc((void**)&tmp, fbytes), "hipMalloc(wall conversion)");
  if (st != LBM_OK) return st;
  c->ops.exp(c->kp, c->pops[c->cur], tmp, c->stream);
  st = hip_check(hipGetLastError(), "export launch");
  if (st == LBM_OK && solid) {
    unsigned* bits = new (std::nothrow) unsigned[c->cells];
    if (!bits) st = lbm_fail(LBM_ERR_ARG, "out of host memory");
    if (st == LBM_OK) {
      if (c->prm.lattice == LBM_D2Q9) wall_bits<LBM_D2Q9>(c->prm.nx, c->prm.ny, c->prm.nz, solid, bits);
      else wall_bits<LBM_D3Q19>(c->prm.nx, c->prm.ny, c->prm.nz, solid, bits);
      if (!c->bb) st = hip_check(hipMalloc((void**)&c->bb, sizeof(unsigned) * c->cells), "hipMalloc(walls)");
    }
    if (st == LBM_OK) st = hip_check(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    if (st == LBM_OK)
      st = hip_check(hipMemcpy(c->bb, bits, sizeof(unsigned) * c->cells, hipMemcpyHostToDevice), "hipMemcpy(walls)");
    delete[] bits;
    if (st == LBM_OK) {
      c->kp.bb = c->bb;
      c->kp.psi_wall = psi_wall;
    }
  } else if (st == LBM_OK) {
    c->kp.bb = nullptr;
    c->kp.psi_wall = 0.0;
  }
  if (st == LBM_OK) {
    c->drop_graphs();   // captured launches hold the old wall arguments
    c->ops.imp(c->kp, c->pops[c->cur], tmp, nullptr, nullptr, 0, c->stream);
    st = hip_check(hipGetLastError(), "import launch");
  }
  const lbm_status st2 = hip_check(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  hipFree(tmp);
  return st != LBM_OK ? st : st2;
}

extern "C" void lbm_destroy(lbm_ctx* c) { delete c; }
