// Launchers of the step and auxiliary kernels, instantiated per (lattice, nc,
// storage, collision, forcing) in the per-lattice translation units.
#pragma once
#include "lbm_adjoint.hpp"

namespace lbmk {

struct Bufs {
  void* p0;   // F64: f;  offset formats: base
  void* p1;   // offset formats: r
  int nc;     // components (the interleaved offset layout's stride)
};

// scratch field of one step: psi
struct StepScratch {
  double* psi;
};

struct Ops {
  void (*psi)(const KParams&, const Bufs&, const StepScratch&, int, int, hipStream_t);
  void (*collide)(const KParams&, const Bufs&, const Bufs&, const StepScratch&, int, int, hipStream_t);
  void (*moments)(const KParams&, const Bufs&, const StepScratch&, double*, double*, double*, double*, double*,
                  hipStream_t);
  void (*exp)(const KParams&, const Bufs&, double*, hipStream_t);
  void (*imp)(const KParams&, const Bufs&, const double*, const double*, const double*, int, hipStream_t);
};

// workgroups for `cells` cells of kBlock threads, rounded to the XCD count
inline int nblocks_for(int cells) { return (int)xcd_grid((cells + kBlock - 1) / kBlock); }

template <int ST>
inline Pops<ST> make_pops(const Bufs& b);
template <>
inline Pops<LBM_F64> make_pops<LBM_F64>(const Bufs& b) {
  Pops<LBM_F64> p;
  p.f = (double*)b.p0;
  return p;
}
template <>
inline Pops<LBM_F32_OFS> make_pops<LBM_F32_OFS>(const Bufs& b) {
  Pops<LBM_F32_OFS> p;
  p.base = (float*)b.p0;
  p.r = (float*)b.p1;
  p.nc = b.nc;
  return p;
}
template <>
inline Pops<LBM_F16_OFS> make_pops<LBM_F16_OFS>(const Bufs& b) {
  Pops<LBM_F16_OFS> p;
  p.base = (float*)b.p0;
  p.r = (__half*)b.p1;
  p.nc = b.nc;
  return p;
}

template <int LAT, int NC, int ST, int COLL, int FORC>
struct OpsImpl {
  // pass 1 over planes [plane0, plane0 + np): k_psi (float64 storage) or k_psi_ilv
  // (interleaved offsets); one-wavefront workgroups on small launches
  template <int B>
  static void psi_launch(const KParams& P, const Bufs& in, double* psi, int plane0, int np, hipStream_t st) {
    constexpr int D = VS<LAT>::D;
    if constexpr (ST == LBM_F64)
      hipLaunchKernelGGL((k_psi<LAT, NC, ST, B>), dim3(psi_blocks(P, np, D, B)), dim3(B), 0, st, P,
                         make_pops<ST>(in), psi, plane0, np);
    else if (P.bb)
      hipLaunchKernelGGL((k_psi_ilv<LAT, NC, ST, B, true>), dim3(psi_blocks(P, np, D, B)), dim3(B), 0, st, P,
                         make_pops<ST>(in), psi, plane0, np);
    else
      hipLaunchKernelGGL((k_psi_ilv<LAT, NC, ST, B, false>), dim3(psi_blocks(P, np, D, B)), dim3(B), 0, st, P,
                         make_pops<ST>(in), psi, plane0, np);
  }
  static void psi(const KParams& P, const Bufs& in, const StepScratch& sc, int plane0, int np, hipStream_t st) {
    if (psi_small(P, np, VS<LAT>::D)) psi_launch<64>(P, in, sc.psi, plane0, np, st);
    else psi_launch<kBlock>(P, in, sc.psi, plane0, np, st);
  }
  static void collide(const KParams& P, const Bufs& in, const Bufs& out, const StepScratch& sc, int plane0,
                      int np, hipStream_t st) {
    // 64-cell segments of the rows (y, z) of the slab
    const int rows = np * (VS<LAT>::D == 3 ? P.ny : 1);
    const int segs = rows * ((P.nx + kCells - 1) / kCells);
    if constexpr (ST == LBM_F64) {   // one workgroup (nc wavefronts) per segment
      hipLaunchKernelGGL((k_collide<LAT, NC, ST, COLL, FORC>), dim3(xcd_grid(segs)), dim3(kCells * NC), 0, st, P,
                         make_pops<ST>(in), make_pops<ST>(out), (const double*)sc.psi, plane0, np);
    } else {                         // ilv_waves segments per workgroup, one per wavefront
      if (P.bb) {
        constexpr int w = ilv_waves(true);
        hipLaunchKernelGGL((k_collide_ilv<LAT, NC, ST, COLL, FORC, true>), dim3(xcd_grid((segs + w - 1) / w)),
                           dim3(64 * w), 0, st, P, make_pops<ST>(in), make_pops<ST>(out), (const double*)sc.psi,
                           plane0, np);
      } else {
        constexpr int w = ilv_waves(false);
        hipLaunchKernelGGL((k_collide_ilv<LAT, NC, ST, COLL, FORC, false>), dim3(xcd_grid((segs + w - 1) / w)),
                           dim3(64 * w), 0, st, P, make_pops<ST>(in), make_pops<ST>(out), (const double*)sc.psi,
                           plane0, np);
      }
    }
  }
  static void moments(const KParams& P, const Bufs& in, const StepScratch& sc, double* rho, double* u, double* p,
                      double* psi_out, double* partials, hipStream_t st) {
    const int nb = nblocks_for(P.cells);
    psi_launch<kBlock>(P, in, sc.psi, 0, P.nplanes, st);
    hipLaunchKernelGGL((k_moments<LAT, NC, ST>), dim3(nb), dim3(kBlock), 0, st, P, make_pops<ST>(in),
                       (const double*)sc.psi, rho, u, p, psi_out, partials);
  }
  static void exp(const KParams& P, const Bufs& in, double* f, hipStream_t st) {
    hipLaunchKernelGGL((k_export<LAT, NC, ST>), dim3(nblocks_for(P.cells)), dim3(kBlock), 0, st, P,
                       make_pops<ST>(in), f);
  }
  static void imp(const KParams& P, const Bufs& out, const double* f, const double* rho0, const double* u0, int mode,
                  hipStream_t st) {
    hipLaunchKernelGGL((k_import<LAT, NC, ST>), dim3(nblocks_for(P.cells)), dim3(kBlock), 0, st, P,
                       make_pops<ST>(out), f, rho0, u0, mode);
  }
  static Ops ops() { return Ops{&psi, &collide, &moments, &exp, &imp}; }
};

template <int LAT, int NC, int ST>
Ops ops_cf(int coll, int forc) {
  if (coll == LBM_BGK) {
    return forc == LBM_GUO ? OpsImpl<LAT, NC, ST, LBM_BGK, LBM_GUO>::ops() : OpsImpl<LAT, NC, ST, LBM_BGK, LBM_EDM>::ops();
  }
  return forc == LBM_GUO ? OpsImpl<LAT, NC, ST, LBM_MRT, LBM_GUO>::ops() : OpsImpl<LAT, NC, ST, LBM_MRT, LBM_EDM>::ops();
}

template <int LAT, int NC>
Ops ops_st(int st, int coll, int forc) {
  switch (st) {
    case LBM_F64: return ops_cf<LAT, NC, LBM_F64>(coll, forc);
    case LBM_F32_OFS: return ops_cf<LAT, NC, LBM_F32_OFS>(coll, forc);
    default: return ops_cf<LAT, NC, LBM_F16_OFS>(coll, forc);
  }
}

template <int LAT>
Ops ops_lat(int nc, int st, int coll, int forc) {
  switch (nc) {
    case 1: return ops_st<LAT, 1>(st, coll, forc);
    case 2: return ops_st<LAT, 2>(st, coll, forc);
    case 3: return ops_st<LAT, 3>(st, coll, forc);
    default: return ops_st<LAT, 4>(st, coll, forc);
  }
}

// Launchers of the adjoint passes and of the loss helpers, per (lattice, nc,
// storage, collision, forcing).
struct AdjOps {
  void (*a)(const KParams&, const Bufs& state, const double* psi, const double* h, const AdjScratch&, hipStream_t);
  void (*b)(const KParams&, const double* psi, const double* h, const AdjScratch&, double* hout, double* partials,
            hipStream_t);
  void (*moles)(const KParams&, const Bufs& state, const unsigned char* mask, double* partials, hipStream_t);
  void (*seed)(const KParams&, const unsigned char* mask, const double* coef, double* h, hipStream_t);
};

template <int LAT, int NC, int ST, int COLL, int FORC>
struct AdjOpsImpl {
  static void a(const KParams& P, const Bufs& state, const double* psi, const double* h, const AdjScratch& S,
                hipStream_t st) {
    hipLaunchKernelGGL((ka_cell<LAT, NC, ST, COLL, FORC>), dim3(adj_blocks(P.cells)), dim3(kAdjBlock), 0, st, P,
                       make_pops<ST>(state), psi, h, S);
  }
  static void b(const KParams& P, const double* psi, const double* h, const AdjScratch& S, double* hout,
                double* partials, hipStream_t st) {
    hipLaunchKernelGGL((kb_cell<LAT, NC, COLL>), dim3(adj_blocks(P.cells)), dim3(kAdjBlock), 0, st, P, psi, h, S,
                       hout, partials);
  }
  static void moles(const KParams& P, const Bufs& state, const unsigned char* mask, double* partials,
                    hipStream_t st) {
    hipLaunchKernelGGL((k_masked_moles<LAT, NC, ST>), dim3(adj_blocks(P.cells)), dim3(kAdjBlock), 0, st, P,
                       make_pops<ST>(state), mask, partials);
  }
  static void seed(const KParams& P, const unsigned char* mask, const double* coef, double* h, hipStream_t st) {
    hipLaunchKernelGGL((k_adj_seed<LAT, NC>), dim3(adj_blocks(P.cells)), dim3(kAdjBlock), 0, st, P, mask, coef[0],
                       coef[1], coef[2], coef[3], h);
  }
  static AdjOps ops() { return AdjOps{&a, &b, &moles, &seed}; }
};

template <int LAT, int NC, int ST>
AdjOps adj_ops_cf(int coll, int forc) {
  if (coll == LBM_BGK)
    return forc == LBM_GUO ? AdjOpsImpl<LAT, NC, ST, LBM_BGK, LBM_GUO>::ops()
                           : AdjOpsImpl<LAT, NC, ST, LBM_BGK, LBM_EDM>::ops();
  return forc == LBM_GUO ? AdjOpsImpl<LAT, NC, ST, LBM_MRT, LBM_GUO>::ops()
                         : AdjOpsImpl<LAT, NC, ST, LBM_MRT, LBM_EDM>::ops();
}

template <int LAT, int NC>
AdjOps adj_ops_st(int st, int coll, int forc) {
  switch (st) {
    case LBM_F64: return adj_ops_cf<LAT, NC, LBM_F64>(coll, forc);
    case LBM_F32_OFS: return adj_ops_cf<LAT, NC, LBM_F32_OFS>(coll, forc);
    default: return adj_ops_cf<LAT, NC, LBM_F16_OFS>(coll, forc);
  }
}

template <int LAT>
AdjOps adj_ops_lat(int nc, int st, int coll, int forc) {
  switch (nc) {
    case 1: return adj_ops_st<LAT, 1>(st, coll, forc);
    case 2: return adj_ops_st<LAT, 2>(st, coll, forc);
    case 3: return adj_ops_st<LAT, 3>(st, coll, forc);
    default: return adj_ops_st<LAT, 4>(st, coll, forc);
  }
}

// defined in lbm_d2q9.hip / lbm_d3q19.hip
Ops ops_d2q9(int nc, int st, int coll, int forc);
Ops ops_d3q19(int nc, int st, int coll, int forc);
AdjOps adj_ops_d2q9(int nc, int st, int coll, int forc);
AdjOps adj_ops_d3q19(int nc, int st, int coll, int forc);

}  // namespace lbmk
