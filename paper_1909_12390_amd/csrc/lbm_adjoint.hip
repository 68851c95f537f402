// C ABI of the discrete adjoint (host side).
//
// lbm_step_adjoint: one reverse step at the context's current state (psi by k_psi,
//   then the two adjoint passes of lbm_adjoint.hpp).
// lbm_adjoint: a loss-gradient run.  Forward nsteps from the current state with a
//   checkpoint of the population state every K steps; the loss of the final
//   state over a cell mask; then, segment by segment from the last, the segment's
//   states are recomputed from its checkpoint (the same two-pass kernels, so they
//   are bitwise the forward's states) and the adjoint is stepped back through
//   them, accumulating the parameter partials in float64 in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "lbm.h"
#include "lbm_ctx.hpp"
#include "lbm_internal.hpp"

namespace lbmk {

// acc[k] += sum over blocks of partials[b][k], in a fixed order (one block)
__global__ __launch_bounds__(kBlock) void k_accumulate(const double* __restrict__ partials, int nblocks, int K,
                                                      double* acc) {
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
    if (threadIdx.x == 0) acc[k] += red[0];
    __syncthreads();
  }
}

__global__ __launch_bounds__(kBlock) void k_zero(double* p, int n) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

}  // namespace lbmk

using namespace lbmk;

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

lbm_status hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) return lbm_fail(LBM_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
  return LBM_OK;
}

size_t storage_bytes(int storage) { return storage == LBM_F64 ? 8 : (storage == LBM_F32_OFS ? 4 : 2); }

// one population state in the context's storage format: [p0 | p1]
struct StateShape {
  size_t p0_bytes, p1_bytes, total;
};
StateShape state_shape(const lbm_ctx* c) {
  StateShape s;
  const size_t nc = (size_t)c->mix.nc;
  if (c->prm.storage == LBM_F64) {
    s.p0_bytes = nc * c->Q * c->cells * 8;
    s.p1_bytes = 0;
    s.total = align_up(s.p0_bytes);
  } else {
    s.p0_bytes = nc * c->cells * 4;
    s.p1_bytes = nc * c->Q * c->cells * storage_bytes(c->prm.storage);
    s.total = align_up(s.p0_bytes) + align_up(s.p1_bytes);
  }
  return s;
}

struct AdjLayout {
  size_t h[2], Fbar, jbar, rbA, rb, partials, acc, ckpt, seg, total;
  int nseg, K, ktheta;
  StateShape st;
};

void adj_layout(const lbm_ctx* c, int nsteps, int K, AdjLayout* L) {
  const size_t cells = c->cells, nc = (size_t)c->mix.nc;
  L->st = state_shape(c);
  L->K = K;
  L->nseg = (nsteps + K - 1) / K;
  L->ktheta = (int)(nc * nc + nc);
  size_t off = 0;
  for (int k = 0; k < 2; ++k) {
    L->h[k] = off;
    off = align_up(off + nc * c->Q * cells * 8);
  }
  L->Fbar = off;
  off = align_up(off + (size_t)c->D * cells * 8);
  L->jbar = off;
  off = align_up(off + (size_t)c->D * cells * 8);
  L->rbA = off;
  off = align_up(off + nc * cells * 8);
  L->rb = off;
  off = align_up(off + nc * cells * 8);
  L->partials = off;
  off = align_up(off + (size_t)adj_blocks((int)cells) * (LBM_MAX_NC * LBM_MAX_NC + LBM_MAX_NC) * 8);
  L->acc = off;
  off = align_up(off + 32 * 8);
  L->ckpt = off;
  off += (size_t)L->nseg * L->st.total;
  L->seg = off;
  off += (size_t)std::max(0, K - 1) * L->st.total;
  L->total = align_up(off);
}

Bufs slot_at(const lbm_ctx* c, char* p, const StateShape& s) {
  Bufs b;
  b.p0 = p;
  b.p1 = c->prm.storage == LBM_F64 ? nullptr : p + align_up(s.p0_bytes);
  b.nc = c->mix.nc;
  return b;
}

lbm_status copy_state(const lbm_ctx* c, const Bufs& dst, const Bufs& src, const StateShape& s) {
  lbm_status st = hip_check(hipMemcpyAsync(dst.p0, src.p0, s.p0_bytes, hipMemcpyDeviceToDevice, c->stream),
                            "copy state");
  if (st == LBM_OK && s.p1_bytes)
    st = hip_check(hipMemcpyAsync(dst.p1, src.p1, s.p1_bytes, hipMemcpyDeviceToDevice, c->stream), "copy state");
  return st;
}

lbm_status supported(const lbm_ctx* c) {
  if (!c) return lbm_fail(LBM_ERR_ARG, "ctx is NULL");
  return LBM_OK;
}

AdjScratch scratch_of(char* ws, const AdjLayout& L) {
  AdjScratch S;
  S.Fbar = (double*)(ws + L.Fbar);
  S.jbar = (double*)(ws + L.jbar);
  S.rbA = (double*)(ws + L.rbA);
  S.rb = (double*)(ws + L.rb);
  return S;
}

// one reverse step at `state`: h (after the step) -> hout (before it); the
// parameter partials are added to the per-block accumulator `partials`
void enqueue_reverse(lbm_ctx* c, const Bufs& state, const double* h, double* hout, const AdjScratch& S,
                     double* partials) {
  c->ops.psi(c->kp, state, c->sc, 0, c->kp.nplanes, c->stream);
  c->adj.a(c->kp, state, c->psi, h, S, c->stream);
  c->adj.b(c->kp, c->psi, h, S, hout, partials, c->stream);
}

void zero(double* p, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_zero, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, p, n);
}

// acc[0..K) = sum over blocks of the per-block accumulator
void finish_partials(const lbm_ctx* c, const double* partials, int K, double* acc) {
  zero(acc, 32, c->stream);
  hipLaunchKernelGGL(k_accumulate, dim3(1), dim3(kBlock), 0, c->stream, partials, adj_blocks((int)c->cells), K,
                     acc);
}

lbm_status read_flag(lbm_ctx* c) {
  int flag = 0;
  lbm_status st = hip_check(hipMemcpyAsync(&flag, c->err, sizeof(int), hipMemcpyDeviceToHost, c->stream),
                            "read error flag");
  if (st == LBM_OK) st = hip_check(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  if (st == LBM_OK && flag) return lbm_fail(LBM_ERR_DOMAIN, "EOS/psi domain violation or non-finite value");
  return st;
}

}  // namespace

extern "C" lbm_status lbm_adjoint_workspace(const lbm_ctx* c, int nsteps, int checkpoint_every, size_t* bytes) {
  if (!c || !bytes || nsteps < 1 || checkpoint_every < 1)
    return lbm_fail(LBM_ERR_ARG, "need ctx, bytes, nsteps >= 1 and checkpoint_every >= 1");
  AdjLayout L;
  adj_layout(c, nsteps, std::min(checkpoint_every, nsteps), &L);
  *bytes = L.total;
  return LBM_OK;
}

extern "C" lbm_status lbm_step_adjoint(lbm_ctx* c, const double* h_next, double* h_out, double* d_aa, double* d_b,
                                       void* ws, size_t ws_bytes) {
  lbm_status st = supported(c);
  if (st != LBM_OK) return st;
  if (!h_next || !h_out || h_next == h_out || !d_aa || !d_b || !ws)
    return lbm_fail(LBM_ERR_ARG, "bad lbm_step_adjoint arguments");
  if ((uintptr_t)ws % kAlign) return lbm_fail(LBM_ERR_ARG, "workspace must be 256-byte aligned");
  AdjLayout L;
  adj_layout(c, 1, 1, &L);
  if (ws_bytes < L.total) return lbm_fail(LBM_ERR_ARG, "workspace too small: %zu < %zu", ws_bytes, L.total);
  char* w = (char*)ws;
  double* acc = (double*)(w + L.acc);
  double* partials = (double*)(w + L.partials);
  const int nb = adj_blocks((int)c->cells);
  zero(partials, nb * L.ktheta, c->stream);
  enqueue_reverse(c, c->pops[c->cur], h_next, h_out, scratch_of(w, L), partials);
  finish_partials(c, partials, L.ktheta, acc);
  st = hip_check(hipGetLastError(), "adjoint launch");
  if (st != LBM_OK) return st;
  double host[LBM_MAX_NC * LBM_MAX_NC + LBM_MAX_NC];
  st = hip_check(hipMemcpyAsync(host, acc, sizeof(double) * L.ktheta, hipMemcpyDeviceToHost, c->stream),
                 "read parameter adjoint");
  if (st == LBM_OK) st = read_flag(c);
  if (st != LBM_OK) return st;
  const int nc = c->mix.nc;
  for (int k = 0; k < nc * nc; ++k) d_aa[k] += host[k];
  for (int i = 0; i < nc; ++i) d_b[i] += host[nc * nc + i];
  return LBM_OK;
}

extern "C" lbm_status lbm_adjoint(lbm_ctx* c, int nsteps, int checkpoint_every, const unsigned char* mask,
                                  const double* x_target, void* ws, size_t ws_bytes, double* loss, double* x_liq,
                                  double* d_k, double* d_a, double* d_b) {
  lbm_status st = supported(c);
  if (st != LBM_OK) return st;
  if (nsteps < 1 || checkpoint_every < 1 || !mask || !x_target || !ws || !loss || !d_k || !d_a || !d_b)
    return lbm_fail(LBM_ERR_ARG, "bad lbm_adjoint arguments");
  if ((uintptr_t)ws % kAlign) return lbm_fail(LBM_ERR_ARG, "workspace must be 256-byte aligned");
  const int K = std::min(checkpoint_every, nsteps);
  AdjLayout L;
  adj_layout(c, nsteps, K, &L);
  if (ws_bytes < L.total) return lbm_fail(LBM_ERR_ARG, "workspace too small: %zu < %zu", ws_bytes, L.total);
  const int nc = c->mix.nc;
  char* w = (char*)ws;
  double* hb[2] = {(double*)(w + L.h[0]), (double*)(w + L.h[1])};
  double* partials = (double*)(w + L.partials);
  double* acc = (double*)(w + L.acc);
  const AdjScratch S = scratch_of(w, L);
  const int nb = adj_blocks((int)c->cells);

  // forward with checkpoints
  for (int s = 0; s < L.nseg && st == LBM_OK; ++s) {
    st = copy_state(c, slot_at(c, w + L.ckpt + (size_t)s * L.st.total, L.st), c->pops[c->cur], L.st);
    if (st == LBM_OK) st = lbm_step(c, std::min(K, nsteps - s * K));
  }
  if (st != LBM_OK) return st;
  st = read_flag(c);
  if (st != LBM_OK) return st;

  // loss over the mask: N_i = sum rbar_i / M_i, x = N / sum N, L = sum (x - x_tgt)^2
  c->adj.moles(c->kp, c->pops[c->cur], mask, partials, c->stream);
  finish_partials(c, partials, nc, acc);
  double Nm[LBM_MAX_NC];
  st = hip_check(hipMemcpyAsync(Nm, acc, sizeof(double) * nc, hipMemcpyDeviceToHost, c->stream), "read moles");
  if (st == LBM_OK) st = hip_check(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  if (st != LBM_OK) return st;
  double Ntot = 0.0;
  for (int i = 0; i < nc; ++i) Ntot += Nm[i];
  if (!(Ntot > 0.0)) return lbm_fail(LBM_ERR_ARG, "the mask holds no moles");
  double x[LBM_MAX_NC], L2 = 0.0;
  for (int i = 0; i < nc; ++i) {
    x[i] = Nm[i] / Ntot;
    L2 += (x[i] - x_target[i]) * (x[i] - x_target[i]);
  }
  *loss = L2;
  if (x_liq)
    for (int i = 0; i < nc; ++i) x_liq[i] = x[i];
  double coef[LBM_MAX_NC] = {0.0, 0.0, 0.0, 0.0};
  for (int k = 0; k < nc; ++k) {
    double g = 0.0;
    for (int i = 0; i < nc; ++i) g += 2.0 * (x[i] - x_target[i]) * ((i == k ? 1.0 : 0.0) - x[i]) / Ntot;
    coef[k] = g / c->mix.M[k];
  }
  c->adj.seed(c->kp, mask, coef, hb[0], c->stream);
  zero(partials, nb * L.ktheta, c->stream);

  // reverse, segment by segment
  int cur = 0;
  for (int s = L.nseg - 1; s >= 0 && st == LBM_OK; --s) {
    const int n = std::min(K, nsteps - s * K);
    auto slot = [&](int i) {
      return i == 0 ? slot_at(c, w + L.ckpt + (size_t)s * L.st.total, L.st)
                    : slot_at(c, w + L.seg + (size_t)(i - 1) * L.st.total, L.st);
    };
    for (int i = 0; i + 1 < n; ++i) {
      const Bufs in = slot(i), out = slot(i + 1);
      c->ops.psi(c->kp, in, c->sc, 0, c->kp.nplanes, c->stream);
      c->ops.collide(c->kp, in, out, c->sc, 0, c->kp.nplanes, c->stream);
    }
    for (int i = n - 1; i >= 0; --i) {
      enqueue_reverse(c, slot(i), hb[cur], hb[1 - cur], S, partials);
      cur = 1 - cur;
    }
    st = hip_check(hipGetLastError(), "adjoint launch");
  }
  if (st != LBM_OK) return st;
  finish_partials(c, partials, L.ktheta, acc);
  double host[LBM_MAX_NC * LBM_MAX_NC + LBM_MAX_NC];
  st = hip_check(hipMemcpyAsync(host, acc, sizeof(double) * L.ktheta, hipMemcpyDeviceToHost, c->stream),
                 "read parameter adjoint");
  if (st == LBM_OK) st = read_flag(c);
  if (st != LBM_OK) return st;
  return lbm_eos_param_grad(&c->mix, c->prm.T, host, host + nc * nc, d_k, d_a, d_b);
}
