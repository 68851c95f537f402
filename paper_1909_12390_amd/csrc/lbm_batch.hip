// C ABI of the batched step: many independent periodic boxes advanced together.
// Each pass of a step is one persistent launch over the (box, tile) work list
// (lbm_batch.hpp); K steps can be captured once in a HIP graph per buffer parity
// and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "lbm.h"
#include "lbm_batch_dispatch.hpp"
#include "lbm_internal.hpp"
#include "lbm_walls.hpp"

using namespace lbmk;

namespace {

lbm_status hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) return lbm_fail(LBM_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
  return LBM_OK;
}

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }
size_t storage_bytes(int storage) { return storage == LBM_F64 ? 8 : (storage == LBM_F32_OFS ? 4 : 2); }

struct BLayout {
  size_t pop0[2], pop1[2], psi, boxes, tiles, fld, err, walls, total;
  size_t field_elems, pop_elems, cells, wall_cells;
  unsigned ntiles;
};

lbm_status batch_validate(const lbm_box* boxes, int nboxes, const lbm_batch_params* prm) {
  if (!boxes || nboxes < 1 || !prm) return lbm_fail(LBM_ERR_ARG, "need boxes, nboxes >= 1 and params");
  if (prm->lattice != LBM_D2Q9 && prm->lattice != LBM_D3Q19) return lbm_fail(LBM_ERR_ARG, "unknown lattice");
  if (prm->collision != LBM_BGK && prm->collision != LBM_MRT) return lbm_fail(LBM_ERR_ARG, "unknown collision");
  if (prm->forcing != LBM_GUO && prm->forcing != LBM_EDM) return lbm_fail(LBM_ERR_ARG, "unknown forcing");
  if (prm->storage < LBM_F64 || prm->storage > LBM_F16_OFS) return lbm_fail(LBM_ERR_ARG, "unknown storage");
  const int t = prm->tile;
  if (!(t == 0 || t == 64 || t == 128 || t == 256)) return lbm_fail(LBM_ERR_ARG, "tile must be 0, 64, 128 or 256");
  if (prm->graph_steps < 0 || prm->grid < 0) return lbm_fail(LBM_ERR_ARG, "graph_steps and grid must be >= 0");
  if (prm->fused != 0 && prm->fused != 1) return lbm_fail(LBM_ERR_ARG, "fused must be 0 or 1");
  if (prm->fused && (prm->lattice != LBM_D2Q9 || prm->storage == LBM_F64))
    return lbm_fail(LBM_ERR_ARG, "the fused step needs D2Q9 and float32 or float16 offset storage");
  const int Q = prm->lattice == LBM_D2Q9 ? 9 : 19;
  if (prm->collision == LBM_MRT)
    for (int k = 0; k < Q; ++k)
      if (!(prm->mrt_s[k] >= 0.0 && prm->mrt_s[k] < 2.0)) return lbm_fail(LBM_ERR_ARG, "MRT rate %d outside [0, 2)", k);
  for (int i = 0; i < nboxes; ++i) {
    const lbm_box& B = boxes[i];
    const lbm_mixture& m = B.mix;
    if (m.nc < 1 || m.nc > LBM_MAX_NC) return lbm_fail(LBM_ERR_ARG, "box %d: nc must be in 1..4", i);
    if (B.nx < 1 || B.ny < 1 || B.nz < 1) return lbm_fail(LBM_ERR_ARG, "box %d: sides must be >= 1", i);
    if (prm->lattice == LBM_D2Q9 && B.nz != 1) return lbm_fail(LBM_ERR_ARG, "box %d: D2Q9 needs nz == 1", i);
    if (prm->fused && B.nx > LBM_FUSED_MAX_NX)
      return lbm_fail(LBM_ERR_ARG, "box %d: the fused step takes rows of at most %d cells", i, LBM_FUSED_MAX_NX);
    // a box's population planes are addressed with 32-bit byte offsets: one
    // component's planes (float64), all components' interleaved planes (offsets)
    const double sb = prm->storage == LBM_F64 ? 8.0 : (prm->storage == LBM_F32_OFS ? 4.0 : 2.0);
    const double span = (double)B.nx * B.ny * B.nz * Q * (prm->storage == LBM_F64 ? 8.0 : sb * m.nc);
    if (span >= 4294967295.0)
      return lbm_fail(LBM_ERR_ARG, "box %d too large: its population planes must stay below 4 GiB", i);
    if (!(B.tau > 0.5) || !(B.G < 0.0) || !(B.T > 0.0) || !std::isfinite(B.beta) || !(m.R > 0.0))
      return lbm_fail(LBM_ERR_ARG, "box %d: need tau > 0.5, G < 0, T > 0, finite beta, R > 0", i);
    if (B.solid && !(std::isfinite(B.psi_wall) && B.psi_wall >= 0.0))
      return lbm_fail(LBM_ERR_ARG, "box %d: psi_wall must be finite and >= 0", i);
    for (int a = 0; a < m.nc; ++a) {
      if (!(B.gamma[a] > 0.0 && B.gamma[a] <= 1.0)) return lbm_fail(LBM_ERR_ARG, "box %d: gamma outside (0, 1]", i);
      if (!(m.a[a] > 0.0 && m.b[a] > 0.0 && m.M[a] > 0.0)) return lbm_fail(LBM_ERR_ARG, "box %d: a, b, M > 0", i);
      for (int b = 0; b < m.nc; ++b)
        if (m.k[a][b] != m.k[b][a]) return lbm_fail(LBM_ERR_ARG, "box %d: k must be symmetric", i);
    }
  }
  return LBM_OK;
}

void batch_layout(const lbm_box* boxes, int nboxes, const lbm_batch_params* prm, BLayout* L) {
  const int Q = prm->lattice == LBM_D2Q9 ? 9 : 19;
  const int tile = prm->tile ? prm->tile : 256;
  L->field_elems = 0;
  L->pop_elems = 0;
  L->cells = 0;
  L->wall_cells = 0;
  L->ntiles = 0;
  for (int i = 0; i < nboxes; ++i) {
    const size_t cells = (size_t)boxes[i].nx * boxes[i].ny * boxes[i].nz;
    L->cells += cells;
    if (boxes[i].solid) L->wall_cells += cells;
    L->field_elems += (size_t)boxes[i].mix.nc * cells;
    L->pop_elems += (size_t)boxes[i].mix.nc * Q * cells;
    L->ntiles += (unsigned)((cells + tile - 1) / tile);
  }
  const size_t s = storage_bytes(prm->storage);
  size_t off = 0;
  for (int k = 0; k < 2; ++k) {
    if (prm->storage == LBM_F64) {
      L->pop0[k] = off;
      off = align_up(off + L->pop_elems * 8);
      L->pop1[k] = 0;
    } else {
      L->pop0[k] = off;
      off = align_up(off + L->field_elems * 4);
      L->pop1[k] = off;
      off = align_up(off + L->pop_elems * s);
    }
  }
  L->psi = off;
  off = align_up(off + L->cells * 8);
  L->boxes = off;
  off = align_up(off + (size_t)nboxes * sizeof(BoxK));
  L->tiles = off;
  off = align_up(off + (size_t)L->ntiles * sizeof(int));
  L->fld = off;
  off = align_up(off + (size_t)nboxes * sizeof(unsigned long long));
  L->err = off;
  off = align_up(off + (size_t)(nboxes + 1) * sizeof(int));
  L->walls = off;                      // masks of the boxes with walls, in box order
  off = align_up(off + L->wall_cells * sizeof(unsigned));
  L->total = off;
}

template <int LAT>
void fill_mrt_b(const lbm_batch_params* prm, BatchK* K) {
  K->mrt_rows = 0;
  for (int k = 0; k < VS<LAT>::Q; ++k) {
    K->mrt_c[k] = (1.0 - prm->mrt_s[k]) / mrow_norm2<LAT>(k);
    if (K->mrt_c[k] != 0.0) K->mrt_rows |= 1u << k;
  }
}

}  // namespace

struct lbm_batch {
  int nboxes;
  std::vector<int> box_nc;
  lbm_batch_params prm;
  BatchK K;
  BOps ops;
  int grid;           // persistent grid of the one-thread-per-cell kernels
  int grid_collide;   // persistent grid of kb_collide
  int grid_step;      // persistent grid of the fused step (fused batches)
  size_t step_lds;    // its LDS bytes per workgroup
  hipStream_t stream;
  BBufs pops[2];
  double* psi;
  unsigned long long* fld_off;
  int* err;
  int cur;
  hipGraphExec_t graph[2];
  int graph_steps;
};

namespace {
void enqueue_batch_step(lbm_batch* b) {
  const BBufs& in = b->pops[b->cur];
  const BBufs& out = b->pops[1 - b->cur];
  if (b->prm.fused) {
    b->ops.step(b->K, b->grid_step, b->step_lds, in, out, b->stream);
  } else {
    b->ops.psi(b->K, b->grid, in, b->psi, b->stream);
    b->ops.collide(b->K, b->grid_collide, in, out, b->psi, b->stream);
  }
  b->cur = 1 - b->cur;
}
}  // namespace

extern "C" lbm_status lbm_batch_layout(const lbm_box* boxes, int nboxes, const lbm_batch_params* prm,
                                       size_t* workspace_bytes, size_t* field_elems, size_t* pop_elems) {
  lbm_status st = batch_validate(boxes, nboxes, prm);
  if (st != LBM_OK) return st;
  BLayout L;
  batch_layout(boxes, nboxes, prm, &L);
  if (workspace_bytes) *workspace_bytes = L.total;
  if (field_elems) *field_elems = L.field_elems;
  if (pop_elems) *pop_elems = L.pop_elems;
  return LBM_OK;
}

extern "C" lbm_status lbm_batch_init(const lbm_box* boxes, int nboxes, const lbm_batch_params* prm, void* ws,
                                     size_t ws_bytes, const double* rho0, void* stream, lbm_batch** out) {
  if (!out) return lbm_fail(LBM_ERR_ARG, "out is NULL");
  *out = nullptr;
  lbm_status st = batch_validate(boxes, nboxes, prm);
  if (st != LBM_OK) return st;
  if (!ws || ((uintptr_t)ws % kAlign) != 0) return lbm_fail(LBM_ERR_ARG, "workspace must be 256-byte aligned");
  if (!rho0) return lbm_fail(LBM_ERR_ARG, "rho0 is NULL");
  BLayout L;
  batch_layout(boxes, nboxes, prm, &L);
  if (ws_bytes < L.total) return lbm_fail(LBM_ERR_ARG, "workspace too small: %zu < %zu", ws_bytes, L.total);

  const int Q = prm->lattice == LBM_D2Q9 ? 9 : 19;
  const int tile = prm->tile ? prm->tile : 256;
  std::vector<BoxK> hb(nboxes);
  std::vector<int> tiles;
  std::vector<unsigned long long> fld(nboxes);
  std::vector<unsigned> bits(L.wall_cells);
  tiles.reserve(L.ntiles);
  unsigned long long pop_off = 0, base_off = 0, psi_off = 0, fo = 0, bb_off = 0;
  for (int i = 0; i < nboxes; ++i) {
    const lbm_box& B = boxes[i];
    BoxK& k = hb[i];
    std::memset(&k, 0, sizeof(k));
    k.nx = B.nx;
    k.ny = B.ny;
    k.nz = B.nz;
    k.nc = B.mix.nc;
    k.cells = (unsigned)((size_t)B.nx * B.ny * B.nz);
    k.first_tile = (unsigned)tiles.size();
    k.pop_off = pop_off;
    k.base_off = base_off;
    k.psi_off = psi_off;
    k.RT = B.mix.R * B.T;
    k.G = B.G;
    k.beta = B.beta;
    k.omega = 1.0 / B.tau;
    double aa[LBM_MAX_NC];
    lbm_internal_aalpha(&B.mix, B.T, aa);
    for (int a = 0; a < k.nc; ++a) {
      k.b[a] = B.mix.b[a];
      k.invM[a] = 1.0 / B.mix.M[a];
      k.gamma[a] = B.gamma[a];
      for (int c = 0; c < k.nc; ++c) k.aa[a][c] = std::sqrt(aa[a] * aa[c]) * (1.0 - B.mix.k[a][c]);
    }
    if (B.solid) {
      k.walls = 1;
      k.bb_off = bb_off;
      k.psi_wall = B.psi_wall;
      if (prm->lattice == LBM_D2Q9) wall_bits<LBM_D2Q9>(B.nx, B.ny, B.nz, B.solid, bits.data() + bb_off);
      else wall_bits<LBM_D3Q19>(B.nx, B.ny, B.nz, B.solid, bits.data() + bb_off);
      bb_off += k.cells;
    }
    const unsigned nt = (k.cells + tile - 1) / tile;
    for (unsigned t = 0; t < nt; ++t) tiles.push_back(i);
    fld[i] = fo;
    fo += (unsigned long long)k.nc * k.cells;
    pop_off += (unsigned long long)k.nc * Q * k.cells;
    base_off += (unsigned long long)k.nc * k.cells;
    psi_off += k.cells;
  }

  lbm_batch* b = new (std::nothrow) lbm_batch();
  if (!b) return lbm_fail(LBM_ERR_ARG, "out of host memory");
  b->prm = *prm;
  b->nboxes = nboxes;
  b->box_nc.resize(nboxes);
  for (int i = 0; i < nboxes; ++i) b->box_nc[i] = boxes[i].mix.nc;
  b->stream = (hipStream_t)stream;
  char* base = (char*)ws;
  for (int k = 0; k < 2; ++k) {
    b->pops[k].p0 = base + L.pop0[k];
    b->pops[k].p1 = prm->storage == LBM_F64 ? nullptr : base + L.pop1[k];
  }
  b->psi = (double*)(base + L.psi);
  b->fld_off = (unsigned long long*)(base + L.fld);
  b->err = (int*)(base + L.err);
  b->cur = 0;
  b->graph[0] = b->graph[1] = nullptr;
  b->graph_steps = prm->graph_steps > 0 ? (prm->graph_steps + 1) / 2 * 2 : 0;   // even: parity preserved
  std::memset(&b->K, 0, sizeof(b->K));
  b->K.boxes = (const BoxK*)(base + L.boxes);
  b->K.tile_box = (const int*)(base + L.tiles);
  b->K.ntiles = L.ntiles;
  b->K.tile = tile;
  b->K.collision = prm->collision;
  b->K.forcing = prm->forcing;
  if (prm->collision == LBM_MRT) {
    if (prm->lattice == LBM_D2Q9) fill_mrt_b<LBM_D2Q9>(prm, &b->K);
    else fill_mrt_b<LBM_D3Q19>(prm, &b->K);
  }
  const int D = prm->lattice == LBM_D2Q9 ? 2 : 3;
  for (int d = 0; d < 3; ++d) b->K.accel[d] = d < D ? prm->accel[d] : 0.0;
  b->K.err = b->err;
  b->K.bb = L.wall_cells ? (const unsigned*)(base + L.walls) : nullptr;
  int ncmax = 1;
  for (int i = 0; i < nboxes; ++i) ncmax = std::max(ncmax, boxes[i].mix.nc);
  b->ops = prm->lattice == LBM_D2Q9 ? bops_d2q9(prm->storage, prm->collision, prm->forcing, ncmax)
                                    : bops_d3q19(prm->storage, prm->collision, prm->forcing, ncmax);

  // persistent grids: resident workgroups (or the caller's choice), a multiple of the XCD count
  int grids[2] = {prm->grid, prm->grid};
  if (prm->grid <= 0) {
    int dev = 0, cus = 0, per_cu[2] = {1, 1};
    st = hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (st == LBM_OK) st = hip_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "cus");
    if (st != LBM_OK) {
      delete b;
      return st;
    }
    b->ops.occupancy(tile, per_cu);
    grids[0] = cus * per_cu[0];
    grids[1] = cus * per_cu[1];
  }
  for (int k = 0; k < 2; ++k) grids[k] = (int)xcd_grid((unsigned)std::max(1, std::min<int>(grids[k], (int)L.ntiles)));
  b->grid = grids[0];
  b->grid_collide = grids[1];
  b->grid_step = 0;
  b->step_lds = 0;
  if (prm->fused) {
    int nx_max = 1;
    for (int i = 0; i < nboxes; ++i) nx_max = std::max(nx_max, boxes[i].nx);
    b->step_lds = fused_lds_bytes(tile, nx_max);
    int g = prm->grid;
    if (g <= 0) {
      int dev = 0, cus = 0, per_cu = 1;
      st = hip_check(hipGetDevice(&dev), "hipGetDevice");
      if (st == LBM_OK) st = hip_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "cus");
      if (st != LBM_OK) {
        delete b;
        return st;
      }
      b->ops.step_occupancy(tile, b->step_lds, &per_cu);
      g = cus * per_cu;
    }
    b->grid_step = (int)xcd_grid((unsigned)std::max(1, std::min<int>(g, (int)L.ntiles)));
  }

  st = hip_check(hipMemcpyAsync((void*)b->K.boxes, hb.data(), hb.size() * sizeof(BoxK), hipMemcpyHostToDevice,
                                b->stream), "upload boxes");
  if (st == LBM_OK)
    st = hip_check(hipMemcpyAsync((void*)b->K.tile_box, tiles.data(), tiles.size() * sizeof(int),
                                  hipMemcpyHostToDevice, b->stream), "upload work list");
  if (st == LBM_OK)
    st = hip_check(hipMemcpyAsync(b->fld_off, fld.data(), fld.size() * sizeof(unsigned long long),
                                  hipMemcpyHostToDevice, b->stream), "upload offsets");
  if (st == LBM_OK && L.wall_cells)
    st = hip_check(hipMemcpyAsync((void*)b->K.bb, bits.data(), bits.size() * sizeof(unsigned), hipMemcpyHostToDevice,
                                  b->stream), "upload wall masks");
  if (st == LBM_OK)
    st = hip_check(hipMemsetAsync(b->err, 0, (size_t)(nboxes + 1) * sizeof(int), b->stream), "clear error flags");
  if (st == LBM_OK) {
    b->ops.init(b->K, b->grid, b->pops[0], b->fld_off, rho0, b->stream);
    st = hip_check(hipGetLastError(), "init launch");
  }
  // the host tables above go out of scope: wait for the uploads
  if (st == LBM_OK) st = hip_check(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
  if (st != LBM_OK) {
    delete b;
    return st;
  }
  *out = b;
  return LBM_OK;
}

extern "C" lbm_status lbm_batch_step(lbm_batch* b, int nsteps) {
  if (!b || nsteps < 0) return lbm_fail(LBM_ERR_ARG, "bad lbm_batch_step arguments");
  int left = nsteps;
  if (b->graph_steps > 0) {
    while (left >= b->graph_steps) {
      const int p = b->cur;
      if (!b->graph[p]) {
        hipGraph_t g = nullptr;
        lbm_status st = hip_check(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), "begin capture");
        if (st != LBM_OK) return st;
        for (int i = 0; i < b->graph_steps; ++i) enqueue_batch_step(b);
        st = hip_check(hipStreamEndCapture(b->stream, &g), "end capture");
        if (st != LBM_OK) return st;
        st = hip_check(hipGraphInstantiate(&b->graph[p], g, nullptr, nullptr, 0), "instantiate graph");
        hipGraphDestroy(g);
        if (st != LBM_OK) return st;
        b->cur = p;   // capture only recorded the launches; replay below performs them
      }
      lbm_status st = hip_check(hipGraphLaunch(b->graph[p], b->stream), "graph launch");
      if (st != LBM_OK) return st;
      b->cur = p;   // an even number of steps keeps the buffer parity
      left -= b->graph_steps;
    }
  }
  for (int i = 0; i < left; ++i) enqueue_batch_step(b);
  return hip_check(hipGetLastError(), "batch step launch");
}

extern "C" lbm_status lbm_batch_fields(lbm_batch* b, double* rho, double* f) {
  if (!b) return lbm_fail(LBM_ERR_ARG, "batch is NULL");
  if (!rho && !f) return LBM_OK;
  b->ops.exp(b->K, b->grid, b->pops[b->cur], b->fld_off, rho, f, b->stream);
  return hip_check(hipGetLastError(), "export launch");
}

extern "C" lbm_status lbm_batch_check(lbm_batch* b) {
  if (!b) return lbm_fail(LBM_ERR_ARG, "batch is NULL");
  lbm_status st = hip_check(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
  if (st != LBM_OK) return st;
  int flag = 0;
  st = hip_check(hipMemcpy(&flag, b->err, sizeof(int), hipMemcpyDeviceToHost), "read error flag");
  if (st != LBM_OK) return st;
  if (flag) return lbm_fail(LBM_ERR_DOMAIN, "EOS/psi domain violation or non-finite value in a box");
  return LBM_OK;
}

extern "C" lbm_status lbm_batch_set_gamma(lbm_batch* b, int box, const double* gamma) {
  if (!b || !gamma || box < 0 || box >= b->nboxes) return lbm_fail(LBM_ERR_ARG, "bad lbm_batch_set_gamma arguments");
  const int nc = b->box_nc[box];
  double g[LBM_MAX_NC] = {0.0, 0.0, 0.0, 0.0};
  for (int i = 0; i < nc; ++i) {
    if (!(gamma[i] > 0.0 && gamma[i] <= 1.0)) return lbm_fail(LBM_ERR_ARG, "gamma_%d outside (0, 1]", i);
    g[i] = gamma[i];
  }
  // the box table lives on the device and is read by every launch (graph replays too):
  // write it in stream order, then wait so the host buffer may go
  BoxK* dst = const_cast<BoxK*>(b->K.boxes) + box;
  lbm_status st = hip_check(hipMemcpyAsync(dst->gamma, g, sizeof(double) * LBM_MAX_NC, hipMemcpyHostToDevice,
                                           b->stream), "update gamma");
  if (st == LBM_OK) st = hip_check(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
  return st;
}

extern "C" lbm_status lbm_batch_box_errors(lbm_batch* b, int* flags) {
  if (!b || !flags) return lbm_fail(LBM_ERR_ARG, "bad lbm_batch_box_errors arguments");
  lbm_status st = hip_check(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
  if (st != LBM_OK) return st;
  return hip_check(hipMemcpy(flags, b->err + 1, (size_t)b->nboxes * sizeof(int), hipMemcpyDeviceToHost),
                   "read box error flags");
}

extern "C" void lbm_batch_destroy(lbm_batch* b) {
  if (!b) return;
  for (int p = 0; p < 2; ++p)
    if (b->graph[p]) hipGraphExecDestroy(b->graph[p]);
  delete b;
}
