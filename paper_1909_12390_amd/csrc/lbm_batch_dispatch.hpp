// Launchers of the batched kernels, instantiated per (lattice, storage,
// collision, forcing, largest component count) in lbm_batch_d2q9.hip and
// lbm_batch_d3q19.hip.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>

#include "lbm_batch.hpp"

namespace lbmk {

struct BBufs {
  void* p0;   // F64: f; offset formats: base
  void* p1;   // offset formats: r
};

template <int ST>
inline BatchPops<ST> bpops(const BBufs& b);
template <>
inline BatchPops<LBM_F64> bpops<LBM_F64>(const BBufs& b) {
  BatchPops<LBM_F64> p;
  p.f = (double*)b.p0;
  return p;
}
template <>
inline BatchPops<LBM_F32_OFS> bpops<LBM_F32_OFS>(const BBufs& b) {
  BatchPops<LBM_F32_OFS> p;
  p.base = (float*)b.p0;
  p.r = (float*)b.p1;
  return p;
}
template <>
inline BatchPops<LBM_F16_OFS> bpops<LBM_F16_OFS>(const BBufs& b) {
  BatchPops<LBM_F16_OFS> p;
  p.base = (float*)b.p0;
  p.r = (__half*)b.p1;
  return p;
}

// grid[0]: the one-thread-per-cell kernels (tile threads); grid[1]: kb_collide
// (ncmax x tile threads)
struct BOps {
  void (*psi)(const BatchK&, int, const BBufs&, double*, hipStream_t);
  void (*collide)(const BatchK&, int, const BBufs&, const BBufs&, const double*, hipStream_t);
  // fused step (kb_step_ilv, D2Q9 offset storage; null otherwise): grid, LDS bytes
  void (*step)(const BatchK&, int, size_t, const BBufs&, const BBufs&, hipStream_t);
  void (*step_occupancy)(int tile, size_t lds, int* per_cu);
  void (*exp)(const BatchK&, int, const BBufs&, const unsigned long long*, double*, double*, hipStream_t);
  void (*init)(const BatchK&, int, const BBufs&, const unsigned long long*, const double*, hipStream_t);
  void (*occupancy)(int tile, int* per_cu);   // resident workgroups per CU: [cell kernels, collide]
  int ncmax;
};

template <int LAT, int NCMAX, int ST, int COLL, int FORC>
struct BOpsImpl {
  // float64: kb_psi / kb_collide (nc_max component groups of tile threads, LDS
  // combine); offset storage: kb_psi_ilv / kb_collide_ilv (tile threads, one cell each)
  static constexpr bool kIlv = ST != LBM_F64;
  static size_t lds(int tile) { return kIlv ? 0 : (size_t)NCMAX * 7 * tile * sizeof(double); }
  static int collide_threads(int tile) { return kIlv ? tile : tile * NCMAX; }
  static void psi(const BatchK& K, int grid, const BBufs& in, double* psi, hipStream_t st) {
    if constexpr (kIlv)
      hipLaunchKernelGGL((kb_psi_ilv<LAT, NCMAX, ST>), dim3(grid), dim3(K.tile), 0, st, K, K.boxes, K.tile_box,
                         bpops<ST>(in), psi);
    else
      hipLaunchKernelGGL((kb_psi<LAT, ST>), dim3(grid), dim3(K.tile), 0, st, K, K.boxes, K.tile_box, bpops<ST>(in),
                         psi);
  }
  static void collide(const BatchK& K, int grid, const BBufs& in, const BBufs& out, const double* psi,
                      hipStream_t st) {
    if constexpr (kIlv)
      hipLaunchKernelGGL((kb_collide_ilv<LAT, NCMAX, ST, COLL, FORC>), dim3(grid), dim3(K.tile), 0, st, K, K.boxes,
                         K.tile_box, bpops<ST>(in), bpops<ST>(out), psi);
    else
      hipLaunchKernelGGL((kb_collide<LAT, NCMAX, ST, COLL, FORC>), dim3(grid), dim3(K.tile * NCMAX), lds(K.tile), st,
                         K, K.boxes, K.tile_box, bpops<ST>(in), bpops<ST>(out), psi);
  }
  static void exp(const BatchK& K, int grid, const BBufs& in, const unsigned long long* off, double* rho,
                  double* f, hipStream_t st) {
    hipLaunchKernelGGL((kb_export<LAT, ST>), dim3(grid), dim3(K.tile), 0, st, K, K.boxes, K.tile_box,
                       bpops<ST>(in), off, rho, f);
  }
  static void init(const BatchK& K, int grid, const BBufs& out, const unsigned long long* off, const double* rho0,
                   hipStream_t st) {
    hipLaunchKernelGGL((kb_init<LAT, ST>), dim3(grid), dim3(K.tile), 0, st, K, K.boxes, K.tile_box,
                       bpops<ST>(out), off, rho0);
  }
  static void occupancy(int tile, int* per_cu) {
    int a = 0, b = 0;
    hipError_t ea, eb;
    if constexpr (kIlv) {
      ea = hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, kb_psi_ilv<LAT, NCMAX, ST>, tile, 0);
      eb = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, kb_collide_ilv<LAT, NCMAX, ST, COLL, FORC>, tile, 0);
    } else {
      ea = hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, kb_psi<LAT, ST>, tile, 0);
      eb = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, kb_collide<LAT, NCMAX, ST, COLL, FORC>, tile * NCMAX,
                                                        lds(tile));
    }
    per_cu[0] = ea == hipSuccess ? std::max(1, a) : 1;
    per_cu[1] = eb == hipSuccess ? std::max(1, b) : 1;
  }
  static constexpr bool kFused = kIlv && LAT == LBM_D2Q9;
  static void step(const BatchK& K, int grid, size_t lds, const BBufs& in, const BBufs& out, hipStream_t st) {
    if constexpr (kFused)
      hipLaunchKernelGGL((kb_step_ilv<LAT, NCMAX, ST, COLL, FORC>), dim3(grid), dim3(K.tile), lds, st, K, K.boxes,
                         K.tile_box, bpops<ST>(in), bpops<ST>(out));
  }
  static void step_occupancy(int tile, size_t lds, int* per_cu) {
    int a = 0;
    hipError_t e = hipErrorInvalidValue;
    if constexpr (kFused)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, kb_step_ilv<LAT, NCMAX, ST, COLL, FORC>, tile, lds);
    *per_cu = e == hipSuccess ? std::max(1, a) : 1;
  }
  static BOps ops() {
    return BOps{&psi, &collide, kFused ? &step : nullptr, kFused ? &step_occupancy : nullptr, &exp, &init, &occupancy,
                NCMAX};
  }
};

template <int LAT, int NCMAX, int ST>
BOps bops_cf(int coll, int forc) {
  if (coll == LBM_BGK)
    return forc == LBM_GUO ? BOpsImpl<LAT, NCMAX, ST, LBM_BGK, LBM_GUO>::ops()
                           : BOpsImpl<LAT, NCMAX, ST, LBM_BGK, LBM_EDM>::ops();
  return forc == LBM_GUO ? BOpsImpl<LAT, NCMAX, ST, LBM_MRT, LBM_GUO>::ops()
                         : BOpsImpl<LAT, NCMAX, ST, LBM_MRT, LBM_EDM>::ops();
}

template <int LAT, int NCMAX>
BOps bops_st(int st, int coll, int forc) {
  switch (st) {
    case LBM_F64: return bops_cf<LAT, NCMAX, LBM_F64>(coll, forc);
    case LBM_F32_OFS: return bops_cf<LAT, NCMAX, LBM_F32_OFS>(coll, forc);
    default: return bops_cf<LAT, NCMAX, LBM_F16_OFS>(coll, forc);
  }
}

template <int LAT>
BOps bops_lat(int st, int coll, int forc, int ncmax) {
  switch (ncmax) {
    case 1: return bops_st<LAT, 1>(st, coll, forc);
    case 2: return bops_st<LAT, 2>(st, coll, forc);
    case 3: return bops_st<LAT, 3>(st, coll, forc);
    default: return bops_st<LAT, 4>(st, coll, forc);
  }
}

BOps bops_d2q9(int st, int coll, int forc, int ncmax);
BOps bops_d3q19(int st, int coll, int forc, int ncmax);

}  // namespace lbmk
