// The context behind the opaque lbm_ctx handle of the C ABI (host side), shared by
// the translation units that implement the step and its adjoint.
#pragma once
#include <hip/hip_runtime.h>

#include "lbm.h"
#include "lbm_dispatch.hpp"

namespace lbmk {

constexpr int kMaxRed = 2 * LBM_MAX_NC + 6;   // reduction width: nc masses + 2 * D + nc negative-density counts

}  // namespace lbmk

struct lbm_ctx {
  lbm_mixture mix;
  lbm_params prm;
  lbmk::KParams kp;
  lbmk::Ops ops;
  lbmk::AdjOps adj;
  int Q, D, K;
  int slab;               // planes per slab (blocked schedule)
  size_t cells;
  hipStream_t stream;
  lbmk::Bufs pops[2];
  lbmk::StepScratch sc;
  double* psi;
  double* partials;
  double* totals;
  int* err;
  int cur;
  int device;             // HIP device current at lbm_init (the workspace's device)
  // OVERLAP schedule: second stream and one event per slab (+ the step boundary)
  hipStream_t aux;
  hipEvent_t* ev;
  int nev;
  // solid walls: per-cell direction mask on the device (kp.bb points here when set)
  unsigned* bb;
  // lbm_step replay: graph_steps (even) steps captured once per buffer parity
  hipGraphExec_t graph[2];
  int graph_steps;
  void drop_graphs() {
    if ((graph[0] || graph[1]) && stream) hipStreamSynchronize(stream);   // no replay in flight
    for (int p = 0; p < 2; ++p) {
      if (graph[p]) hipGraphExecDestroy(graph[p]);
      graph[p] = nullptr;
    }
  }
  ~lbm_ctx() {
    drop_graphs();
    for (int k = 0; k < nev; ++k) hipEventDestroy(ev[k]);
    delete[] ev;
    if (aux) hipStreamDestroy(aux);
    if (bb) hipFree(bb);
  }
};
