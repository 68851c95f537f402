// Batched step: many independent periodic boxes, each with its own mixture,
// temperature, volatility coefficients and component count (1..4), advanced by
// one launch per pass per step over a (box, tile) work list.
//
// Storage: the boxes' population planes are concatenated; box b owns the
// elements [pop_off, pop_off + nc Q cells) of the population array(s) (and
// [base_off, base_off + nc cells) of the float32 base in the offset formats),
// plus [psi_off, psi_off + cells) of the psi scratch.  float64 boxes keep
// per-component planes [nc][Q][cells] (kb_psi / kb_collide); the offset formats
// interleave the components, [Q][cells][nc] (kb_psi_ilv / kb_collide_ilv).  The
// per-step arithmetic is the single-box one (lbm_kernels.hpp), with the
// component count read from the box descriptor.
//
// Launch: a persistent grid (a multiple of the 8 XCDs, sized to the resident
// workgroups); XCD x sweeps tiles [x T/8, (x+1) T/8) of the work list in order, so
// each XCD's L2 sees contiguous cells of the same boxes.  Every workgroup leaves
// its loop after at most ceil(T / gridDim) tiles.
#pragma once
#include "lbm_kernels.hpp"

namespace lbmk {

struct BoxK {
  int nx, ny, nz, nc;
  unsigned cells;
  unsigned first_tile;              // first entry of this box in the work list
  unsigned long long pop_off;       // element offset of the box's populations
  unsigned long long base_off;      // element offset of the box's float32 base (offset formats)
  unsigned long long psi_off;       // element offset of the box's psi
  double RT, G, beta, omega;
  double aa[LBM_MAX_NC][LBM_MAX_NC];
  double b[LBM_MAX_NC], invM[LBM_MAX_NC], gamma[LBM_MAX_NC];
  int walls;                        // the box has solid cells (masks at BatchK::bb + bb_off)
  unsigned long long bb_off;        // element offset of the box's wall masks
  double psi_wall;                  // psi of the box's solid cells
};

// Scalars of a batch; the box table and the work list (box of each tile) are
// passed to the kernels as separate restrict pointers, so that their loads,
// uniform per tile, go through the scalar cache.
struct BatchK {
  const BoxK* boxes;
  const int* tile_box;
  unsigned ntiles;
  int tile;                         // cells per tile (= workgroup size)
  int collision, forcing;
  double mrt_c[LBM_MAX_Q];
  unsigned mrt_rows;                // bit k: mrt_c[k] != 0
  double accel[3];
  int* err;                         // [0]: any box; [1 + b]: box b
  const unsigned* bb;               // wall masks of every box with walls (bit a: the source
                                    // x - e_a is solid; bit 31: the cell is solid), or null
};

// Storage views over a box's planes (same encodings as Pops<ST>).
template <int ST>
struct BatchPops;
template <>
struct BatchPops<LBM_F64> {
  using R = double;
  double* f;
  __device__ __forceinline__ Pops<LBM_F64>::View comp(const BoxK& B, int s, int Q) const {
    const unsigned plane = B.cells * 8u;
    return Pops<LBM_F64>::View{make_rsrc(f + B.pop_off + (size_t)s * Q * B.cells, (unsigned)Q * plane), plane};
  }
};
// Component-interleaved offsets of the boxes (as IlvPops for the single box): box
// b's offsets [Q][cells_b][nc_b] at elements [pop_off, pop_off + nc Q cells) of r,
// its bases [cells_b][nc_b] at [base_off, base_off + nc cells) of base; comp(s)
// views component s (the kernels around the step), bufs() gives the all-component
// planes (kb_psi_ilv, kb_collide_ilv).
template <typename H>
struct BatchIlvPops {
  using R = float;
  using Elem = H;
  float* base;
  H* r;
  using View = typename IlvPops<H>::View;
  __device__ __forceinline__ View comp(const BoxK& B, int s, int Q) const {
    const unsigned cs = (unsigned)B.nc * (unsigned)sizeof(H);
    const unsigned plane = B.cells * cs;
    return View{make_rsrc(base + B.base_off, B.cells * (unsigned)B.nc * 4u), make_rsrc(r + B.pop_off, (unsigned)Q * plane),
                plane, cs, (unsigned)s * (unsigned)sizeof(H), (unsigned)B.nc * 4u, (unsigned)s * 4u};
  }
  template <int NC, int Q>
  __device__ __forceinline__ IlvBufs<H, NC, Q> bufs(const BoxK& B) const {
    return IlvBufs<H, NC, Q>(base + B.base_off, r + B.pop_off, B.cells);
  }
};
template <>
struct BatchPops<LBM_F32_OFS> : BatchIlvPops<float> {};
template <>
struct BatchPops<LBM_F16_OFS> : BatchIlvPops<__half> {};

__device__ __forceinline__ void batch_flag(const BatchK& K, int box) {
  K.err[0] = 1;
  K.err[1 + box] = 1;
}

// tiles of this workgroup: XCD-contiguous ranges of the work list
struct TileRange {
  unsigned t, end, stride;
};
__device__ __forceinline__ TileRange tile_range(unsigned ntiles) {
  const unsigned nb = gridDim.x, b = blockIdx.x;
  const unsigned per_xcd_blocks = nb / kXcd;
  const unsigned x = b % kXcd, i = b / kXcd;
  const unsigned lo = (unsigned)(((unsigned long long)ntiles * x) / kXcd);
  const unsigned hi = (unsigned)(((unsigned long long)ntiles * (x + 1)) / kXcd);
  return TileRange{lo + i, hi, per_xcd_blocks};
}

__device__ __forceinline__ Coord box_coord(unsigned cell, const BoxK& B) {
  KParams P;
  P.nx = B.nx;
  P.ny = B.ny;
  P.nz = B.nz;
  return make_coord(cell, P);
}

// mixture pressure and psi with a runtime component count (rb[i] = 0 for i >= nc)
__device__ __forceinline__ double box_psi(const BatchK& K, const BoxK& B, int box, const double* rb) {
  double n[LBM_MAX_NC];
  double rt = 0.0, Bn = 0.0, rho = 0.0;
#pragma unroll
  for (int i = 0; i < LBM_MAX_NC; ++i) {
    n[i] = i < B.nc ? rb[i] * B.invM[i] : 0.0;
    rt += n[i];
    Bn += (i < B.nc ? B.b[i] : 0.0) * n[i];
    rho += i < B.nc ? rb[i] : 0.0;
  }
  double An = 0.0;
#pragma unroll
  for (int i = 0; i < LBM_MAX_NC; ++i) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < LBM_MAX_NC; ++j)
      if (i < B.nc && j < B.nc) s += B.aa[i][j] * n[j];
    An += n[i] * s;
  }
  const double p = rt * B.RT / (1.0 - Bn) - An / (1.0 + 2.0 * Bn - Bn * Bn);
  const double X = 6.0 * (p - rho * (1.0 / 3.0)) / B.G;
  if (!(Bn < 1.0) || !(X >= 0.0) || !(X <= 1.0e300)) batch_flag(K, box);
  return sqrt(X);
}

// pass 1 over every tile (float64 planes): densities -> EOS -> psi
template <int LAT, int ST>
__global__ __launch_bounds__(1024) void kb_psi(BatchK K, const BoxK* __restrict__ boxes, const int* __restrict__ tile_box,
                                              BatchPops<ST> in, double* __restrict__ psi) {
  static_assert(ST == LBM_F64, "the offset formats use kb_psi_ilv");
  using V = VS<LAT>;
  using R = typename BatchPops<ST>::R;
  const TileRange tr = tile_range(K.ntiles);
  for (unsigned t = tr.t; t < tr.end; t += tr.stride) {
    const int bx = __builtin_amdgcn_readfirstlane(tile_box[t]);
    const BoxK& B = boxes[bx];
    const unsigned cell = (t - B.first_tile) * (unsigned)K.tile + threadIdx.x;
    if (cell >= B.cells) continue;
    const Coord c = box_coord(cell, B);
    const unsigned bits = B.walls ? K.bb[B.bb_off + cell] : 0u;
    if (bits >> kSolidBit) {           // solid cell: the wall's psi
      psi[B.psi_off + cell] = B.psi_wall;
      continue;
    }
    double rb[LBM_MAX_NC];
#pragma unroll
    for (int s = 0; s < LBM_MAX_NC; ++s) rb[s] = 0.0;
#pragma unroll 1
    for (int s = 0; s < B.nc; ++s) {
      const auto cv = in.comp(B, s, V::Q);
      R v[V::Q];
      if (B.walls) {                   // halfway bounce-back for sources that are solid
#pragma unroll
        for (int a = 0; a < V::Q; ++a)
          v[a] = pull_bb<LAT>(cv, a, bits, cell, c.at(-V::cx(a), -V::cy(a), -V::cz(a)), (R)V::w(a));
      } else {
        cv.template get_all<V::Q>([&](int a) { return c.at(-V::cx(a), -V::cy(a), -V::cz(a)); }, v,
                                  [](int a) { return (R)V::w(a); });
      }
      R acc = 0;
#pragma unroll
      for (int a = 0; a < V::Q; ++a) acc += v[a];
#pragma unroll
      for (int u = 0; u < LBM_MAX_NC; ++u)
        if (u == s) rb[u] = (double)acc;
    }
    psi[B.psi_off + cell] = box_psi(K, B, bx, rb);
  }
}

// pass 2 over every tile (float64 planes).  A workgroup is NCMAX groups of `tile` threads (the
// largest component count of the batch); group s owns component s of the tile's
// cells, as in the single-box k_collide: it pulls and decodes that component,
// adds a share of the psi stencil (directions a with (a - 1) mod NCMAX = s, also
// in groups with s >= nc of a box with fewer components), and the groups combine
// densities, momenta and force through LDS in a fixed order before each collides
// its own component.  Dynamic LDS: NCMAX x 7 x tile doubles.
template <int LAT, int NCMAX, int ST, int COLL, int FORC>
__global__ __launch_bounds__(1024) void kb_collide(BatchK K, const BoxK* __restrict__ boxes,
                                                  const int* __restrict__ tile_box, BatchPops<ST> in,
                                                  BatchPops<ST> out, const double* __restrict__ psi) {
  static_assert(ST == LBM_F64, "the offset formats use kb_collide_ilv");
  using V = VS<LAT>;
  using R = typename BatchPops<ST>::R;
  constexpr int Q = V::Q;
  extern __shared__ double kb_red[];   // [NCMAX][7][tile]
  const int tile = K.tile;
  // uniform per wavefront (tile is a multiple of 64)
  const int s = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / (unsigned)tile));
  const int lane = (int)threadIdx.x - s * tile;
  KParams P;
  P.mrt_c[0] = 0.0;
#pragma unroll
  for (int k = 0; k < LBM_MAX_Q; ++k) P.mrt_c[k] = K.mrt_c[k];
  P.mrt_rows = K.mrt_rows;
  const TileRange tr = tile_range(K.ntiles);
  for (unsigned t = tr.t; t < tr.end; t += tr.stride) {
    const int bx = __builtin_amdgcn_readfirstlane(tile_box[t]);
    const BoxK& B = boxes[bx];
    const int nc = B.nc;
    const unsigned cell = (t - B.first_tile) * (unsigned)tile + (unsigned)lane;
    // solid cells (walls) do not pull and do not collide; their slots are never
    // read and hold zeros, which their lanes store again so that the tile's rows
    // are written whole
    const unsigned bits = (B.walls && cell < B.cells) ? K.bb[B.bb_off + cell] : 0u;
    const bool in_box = cell < B.cells && !(bits >> kSolidBit);
    const bool active = in_box && s < nc;
    const bool store = cell < B.cells && s < nc;
    const Coord c = box_coord(cell < B.cells ? cell : 0u, B);
    R f[Q];
    R jx = 0, jy = 0, jz = 0;
    double mass = 0.0;   // summed exactly for the offset formats' base (put_all)
    double Fp[3] = {0.0, 0.0, 0.0};
    if (active) {
      const auto cv = in.comp(B, s, Q);
#pragma unroll
      for (int a = 0; a < Q; ++a) {
        const unsigned nbr = c.at(-V::cx(a), -V::cy(a), -V::cz(a));
        f[a] = B.walls ? pull_bb<LAT>(cv, a, bits, cell, nbr, (R)V::w(a)) : cv.get(a, nbr, (R)V::w(a));
        mass += (double)f[a];
        if (V::cx(a)) jx += (R)V::cx(a) * f[a];
        if (V::cy(a)) jy += (R)V::cy(a) * f[a];
        if (V::cz(a)) jz += (R)V::cz(a) * f[a];
      }
    } else {
#pragma unroll
      for (int a = 0; a < Q; ++a) f[a] = 0;
    }
    if (in_box) {
      const double* ps = psi + B.psi_off;
      const double p0 = ps[cell];
      const double hb = 0.5 * (1.0 - B.beta);
      static_for<1, Q>([&](auto A) {
        constexpr int a = decltype(A)::value;
        if ((a - 1) % NCMAX == s) {
          const double pn = ps[c.at(V::cx(a), V::cy(a), V::cz(a))];
          const double tt = V::w(a) * pn * (B.beta * p0 + hb * pn);
          if constexpr (V::cx(a) != 0) Fp[0] += V::cx(a) * tt;
          if constexpr (V::cy(a) != 0) Fp[1] += V::cy(a) * tt;
          if constexpr (V::cz(a) != 0) Fp[2] += V::cz(a) * tt;
        }
      });
    }
    double* red = kb_red + (size_t)s * 7 * tile;
    red[0 * tile + lane] = mass;
    red[1 * tile + lane] = (double)jx;
    red[2 * tile + lane] = (double)jy;
    red[3 * tile + lane] = (double)jz;
    red[4 * tile + lane] = Fp[0];
    red[5 * tile + lane] = Fp[1];
    red[6 * tile + lane] = Fp[2];
    __syncthreads();
    if (store) {
      double rho = 0.0, Gam = 0.0, j[3] = {0.0, 0.0, 0.0}, F[3] = {0.0, 0.0, 0.0};
#pragma unroll
      for (int q = 0; q < NCMAX; ++q) {
        const double* rq = kb_red + (size_t)q * 7 * tile;
        if (q < nc) {
          const double r = rq[lane];
          rho += r;
          Gam += B.gamma[q] * r;
          j[0] += rq[1 * tile + lane];
          j[1] += rq[2 * tile + lane];
          j[2] += rq[3 * tile + lane];
        }
        F[0] += rq[4 * tile + lane];
        F[1] += rq[5 * tile + lane];
        F[2] += rq[6 * tile + lane];
      }
      F[0] *= -B.G;
      F[1] *= -B.G;
      F[2] *= -B.G;
      if (active && !(Gam > 0.0)) batch_flag(K, bx);
      const R g0 = (R)K.accel[0], g1 = (R)K.accel[1], g2 = (R)K.accel[2];
      const R rhoR = (R)rho, irho = (R)1 / rhoR;
      const R FR[3] = {(R)F[0], (R)F[1], (R)F[2]};
      R u[3];
      const R rs = (R)mass;
      const R ch = (R)B.gamma[s] / (R)Gam;
      if (FORC == LBM_GUO) {
        u[0] = ((R)j[0] + (R)0.5 * (FR[0] + rhoR * g0)) * irho;
        u[1] = ((R)j[1] + (R)0.5 * (FR[1] + rhoR * g1)) * irho;
        u[2] = ((R)j[2] + (R)0.5 * (FR[2] + rhoR * g2)) * irho;
      } else {   // component s relaxes towards U - du_s / 2 (as in k_collide)
        u[0] = ((R)j[0] + (R)0.5 * FR[0]) * irho - (R)0.5 * (ch * FR[0]);
        u[1] = ((R)j[1] + (R)0.5 * FR[1]) * irho - (R)0.5 * (ch * FR[1]);
        u[2] = ((R)j[2] + (R)0.5 * FR[2]) * irho - (R)0.5 * (ch * FR[2]);
      }
      R fs[3];
      if (FORC == LBM_GUO) {
        fs[0] = ch * rs * FR[0] + rs * g0;
        fs[1] = ch * rs * FR[1] + rs * g1;
        fs[2] = ch * rs * FR[2] + rs * g2;
      } else {
        fs[0] = ch * FR[0] + g0;
        fs[1] = ch * FR[1] + g1;
        fs[2] = ch * FR[2] + g2;
      }
      if (!active) {   // a solid cell: f = 0, rbar = 0 and u = du = 0 collide to zeros
        u[0] = u[1] = u[2] = 0;
        fs[0] = fs[1] = fs[2] = 0;
      }
      P.cells = (int)B.cells;
      P.omega = B.omega;
      collide_values<LAT, R, COLL, FORC>(P, f, rs, u, fs, [&](const R* fo) {
        out.comp(B, s, Q).template put_all<Q>(cell, fo, mass, [](int a) { return (R)V::w(a); });
      });
    }
    __syncthreads();   // the LDS rows are reused by the next tile
  }
}

// rbar_s of every cell of every box (concatenated [box][nc_b][cells_b]) and the
// state in the canonical float64 layout [box][nc_b][Q][cells_b] (either may be null)
template <int LAT, int ST>
__global__ __launch_bounds__(1024) void kb_export(BatchK K, const BoxK* __restrict__ boxes,
                                                 const int* __restrict__ tile_box, BatchPops<ST> in,
                                                 const unsigned long long* __restrict__ fld_off,
                                                 double* __restrict__ rho_out, double* __restrict__ f_out) {
  using V = VS<LAT>;
  using R = typename BatchPops<ST>::R;
  const TileRange tr = tile_range(K.ntiles);
  for (unsigned t = tr.t; t < tr.end; t += tr.stride) {
    const int bx = __builtin_amdgcn_readfirstlane(tile_box[t]);
    const BoxK& B = boxes[bx];
    const unsigned cell = (t - B.first_tile) * (unsigned)K.tile + threadIdx.x;
    if (cell >= B.cells) continue;
    const Coord c = box_coord(cell, B);
    const unsigned bits = B.walls ? K.bb[B.bb_off + cell] : 0u;
#pragma unroll 1
    for (int s = 0; s < B.nc; ++s) {
      const auto cv = in.comp(B, s, V::Q);
      double acc = 0.0;
#pragma unroll
      for (int a = 0; a < V::Q; ++a) {
        const unsigned nbr = c.at(-V::cx(a), -V::cy(a), -V::cz(a));
        double v;
        if (!B.walls) v = (double)cv.get(a, nbr, (R)V::w(a));
        else if (bits >> kSolidBit) v = 0.0;   // solid cells hold no fluid
        else v = (double)pull_bb<LAT>(cv, a, bits, cell, nbr, (R)V::w(a));
        acc += v;
        if (f_out) f_out[B.pop_off + ((size_t)s * V::Q + a) * B.cells + cell] = v;
      }
      if (rho_out) rho_out[fld_off[bx] + (size_t)s * B.cells + cell] = acc;
    }
  }
}

// equilibrium initialisation from rho0 (concatenated [box][nc_b][cells_b]) at rest
template <int LAT, int ST>
__global__ __launch_bounds__(1024) void kb_init(BatchK K, const BoxK* __restrict__ boxes,
                                               const int* __restrict__ tile_box, BatchPops<ST> out,
                                               const unsigned long long* __restrict__ fld_off,
                                               const double* __restrict__ rho0) {
  using V = VS<LAT>;
  using R = typename BatchPops<ST>::R;
  constexpr int Q = V::Q;
  const TileRange tr = tile_range(K.ntiles);
  for (unsigned t = tr.t; t < tr.end; t += tr.stride) {
    const int bx = __builtin_amdgcn_readfirstlane(tile_box[t]);
    const BoxK& B = boxes[bx];
    const unsigned cell = (t - B.first_tile) * (unsigned)K.tile + threadIdx.x;
    if (cell >= B.cells) continue;
    const Coord c = box_coord(cell, B);
    const unsigned bits = B.walls ? K.bb[B.bb_off + cell] : 0u;
#pragma unroll 1
    for (int s = 0; s < B.nc; ++s) {
      R v[Q];
      double sum = 0.0;
#pragma unroll
      for (int a = 0; a < Q; ++a) {
        // at rest feq depends on |e| only: a population that will bounce back into
        // this cell (its target y + e_a is solid) is the equilibrium of this cell
        const bool back = (bits >> V::opp(a)) & 1u;
        const unsigned src = back ? cell : c.at(V::cx(a), V::cy(a), V::cz(a));
        const double r = (bits >> kSolidBit) ? 0.0 : rho0[fld_off[bx] + (size_t)s * B.cells + src];
        const double fe = feq<LAT, double>(a, r, 0.0, 0.0, 0.0, 0.0);
        v[a] = (R)fe;
        sum += fe;
      }
      out.comp(B, s, Q).template put_all<Q>(cell, v, sum, [](int a) { return (R)V::w(a); });
    }
  }
}

// ---------------------------------------------------------------------------
// Interleaved offset storage: one cell per thread with all its components (the
// box's component count selects the instantiation, uniform per tile)
// ---------------------------------------------------------------------------

// cache policy of the batched offset loads: float16 keeps the default (a 64-cell
// tile spans several short rows, whose shifted pulls read lines of the
// neighbouring tile again), float32 streams them
template <typename H>
constexpr int kbi_load_policy() { return std::is_same<H, __half>::value ? 0 : kPopLoad; }

template <int LAT, int NC, typename H>
__device__ __forceinline__ void kbi_psi_cell(const BatchK& K, const BoxK& B, int bx, const BatchIlvPops<H>& in,
                                             const Coord& c, unsigned cell, unsigned bits, double* psi) {
  constexpr int Q = VS<LAT>::Q;
  const auto Bf = in.template bufs<NC, Q>(B);
  float f[NC][Q];
  ilv_pull_cell<LAT, NC, H, kbi_load_policy<H>()>(Bf, c, cell, bits, B.walls != 0, f);
  double rb[LBM_MAX_NC];
#pragma unroll
  for (int s = 0; s < LBM_MAX_NC; ++s) rb[s] = 0.0;
#pragma unroll
  for (int s = 0; s < NC; ++s) {
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < Q; ++a) acc += (double)f[s][a];
    rb[s] = acc;
  }
  psi[B.psi_off + cell] = box_psi(K, B, bx, rb);
}

// pass 1 over every tile (interleaved offsets): densities -> EOS -> psi
template <int LAT, int NCMAX, int ST>
__global__ __launch_bounds__(256) void kb_psi_ilv(BatchK K, const BoxK* __restrict__ boxes,
                                                  const int* __restrict__ tile_box, BatchPops<ST> in,
                                                  double* __restrict__ psi) {
  using H = typename BatchPops<ST>::Elem;
  const TileRange tr = tile_range(K.ntiles);
  for (unsigned t = tr.t; t < tr.end; t += tr.stride) {
    const int bx = __builtin_amdgcn_readfirstlane(tile_box[t]);
    const BoxK& B = boxes[bx];
    const unsigned cell = (t - B.first_tile) * (unsigned)K.tile + threadIdx.x;
    if (cell >= B.cells) continue;
    const Coord c = box_coord(cell, B);
    const unsigned bits = B.walls ? K.bb[B.bb_off + cell] : 0u;
    if (bits >> kSolidBit) {           // solid cell: the wall's psi
      psi[B.psi_off + cell] = B.psi_wall;
      continue;
    }
    const int nc = B.nc;
    if (nc == 1) kbi_psi_cell<LAT, 1, H>(K, B, bx, in, c, cell, bits, psi);
    if constexpr (NCMAX >= 2)
      if (nc == 2) kbi_psi_cell<LAT, 2, H>(K, B, bx, in, c, cell, bits, psi);
    if constexpr (NCMAX >= 3)
      if (nc == 3) kbi_psi_cell<LAT, 3, H>(K, B, bx, in, c, cell, bits, psi);
    if constexpr (NCMAX >= 4)
      if (nc == 4) kbi_psi_cell<LAT, 4, H>(K, B, bx, in, c, cell, bits, psi);
  }
}

// The collision of one cell from its pulled populations f (zeros for a solid cell)
// and psi at the cell and its neighbours (pn[a] at x + e_a): the force, the split,
// the collision, the encoding and the stores of the cell's slots.
template <int LAT, int NC, typename H, int COLL, int FORC>
__device__ __forceinline__ void kbi_collide_pulled(const BatchK& K, const KParams& P, const BoxK& B, int bx,
                                                   const BatchIlvPops<H>& out, unsigned cell, bool valid,
                                                   float (&f)[NC][VS<LAT>::Q], const double (&pn)[VS<LAT>::Q]) {
  using V = VS<LAT>;
  using R = float;
  constexpr int Q = V::Q;
  constexpr int NW = IlvWords<H, NC>::N;
  using IB = IlvBufs<H, NC, Q>;
  // total force of Eq. (coupledMCforce) (float64), summed over opposite pairs
  double F[3] = {0.0, 0.0, 0.0};
  {
    const double hb = 0.5 * (1.0 - B.beta);
    const double bps = B.beta * pn[0];
    static_for<0, (Q - 1) / 2>([&](auto Pp) {
      constexpr int a = V::pair_first(decltype(Pp)::value), b = V::opp(a);
      const double t = V::w(a) * (pn[a] - pn[b]) * (bps + hb * (pn[a] + pn[b]));
      if constexpr (V::cx(a) != 0) F[0] += V::cx(a) * t;
      if constexpr (V::cy(a) != 0) F[1] += V::cy(a) * t;
      if constexpr (V::cz(a) != 0) F[2] += V::cz(a) * t;
    });
    F[0] *= -B.G;
    F[1] *= -B.G;
    F[2] *= -B.G;
  }
  double mass[NC], rho = 0.0, Gam = 0.0, j[3];
#pragma unroll
  for (int s = 0; s < NC; ++s) {
    double m = 0.0;
#pragma unroll
    for (int a = 0; a < Q; ++a) m += (double)f[s][a];
    mass[s] = m;
    rho += m;
    Gam += B.gamma[s] * m;
  }
  {
    R jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int a = 1; a < Q; ++a) {
      R g = f[0][a];
#pragma unroll
      for (int s = 1; s < NC; ++s) g += f[s][a];
      if (V::cx(a)) jx += (R)V::cx(a) * g;
      if (V::cy(a)) jy += (R)V::cy(a) * g;
      if (V::cz(a)) jz += (R)V::cz(a) * g;
    }
    j[0] = (double)jx;
    j[1] = (double)jy;
    j[2] = (double)jz;
  }
  if (valid && !(Gam > 0.0)) batch_flag(K, bx);
  unsigned ro[Q][NW];
  float bo[NC];
  static_for<0, NC>([&](auto S_) {
    constexpr int s = decltype(S_)::value;
    const R rs = (R)mass[s];
    R u[3], fs[3];
    cell_velocity_split<FORC>(P, s, rho, Gam, j, F, rs, u, fs);
    if (!valid) {   // a solid cell: f = 0, rbar = 0 and u = du = 0 collide to zeros
      u[0] = u[1] = u[2] = 0;
      fs[0] = fs[1] = fs[2] = 0;
    }
    collide_values<LAT, R, COLL, FORC>(P, f[s], rs, u, fs, [&](const R* fo) {
      H rq[Q];
      bo[s] = encode_offsets<Q, H, true>(fo, mass[s], [](int a) { return (R)V::w(a); }, rq);
#pragma unroll
      for (int a = 0; a < Q; ++a) ilv_set<H>(ro[a], s, rq[a]);
    });
  });
  const IB Bo = out.template bufs<NC, Q>(B);
#pragma unroll
  for (int a = 0; a < Q; ++a) ilv_store<kPopStore, H, NC>(Bo.rr, cell * IB::cs, (unsigned)a * Bo.plane, ro[a]);
  unsigned bw[NC];
#pragma unroll
  for (int s = 0; s < NC; ++s) bw[s] = __builtin_bit_cast(unsigned, bo[s]);
  ilv_store<kBaseStore, float, NC>(Bo.rb, cell * IB::bs, 0u, bw);
}

template <int LAT, int NC, typename H, int COLL, int FORC>
__device__ __forceinline__ void kbi_collide_cell(const BatchK& K, const KParams& P, const BoxK& B, int bx,
                                                 const BatchIlvPops<H>& in, const BatchIlvPops<H>& out,
                                                 const Coord& c, unsigned cell, unsigned bits,
                                                 const double* __restrict__ psi) {
  using V = VS<LAT>;
  constexpr int Q = V::Q;
  const bool valid = !(bits >> kSolidBit);
  const double* ps = psi + B.psi_off;
  double pn[Q];
#pragma unroll
  for (int a = 0; a < Q; ++a) pn[a] = ps[c.at(V::cx(a), V::cy(a), V::cz(a))];
  const auto Bi = in.template bufs<NC, Q>(B);
  float f[NC][Q];
  if (valid) {
    ilv_pull_cell<LAT, NC, H, kbi_load_policy<H>()>(Bi, c, cell, bits, B.walls != 0, f);
  } else {   // solid cells: no pull, no collision; their lanes store zeros into never-read slots
#pragma unroll
    for (int s = 0; s < NC; ++s)
#pragma unroll
      for (int a = 0; a < Q; ++a) f[s][a] = 0.0f;
  }
  kbi_collide_pulled<LAT, NC, H, COLL, FORC>(K, P, B, bx, out, cell, valid, f, pn);
}

// pass 2 over every tile (interleaved offsets): one cell per thread with all its
// components (no LDS, no idle component groups for boxes with fewer components)
template <int LAT, int NCMAX, int ST, int COLL, int FORC>
__global__ __launch_bounds__(256) void kb_collide_ilv(BatchK K, const BoxK* __restrict__ boxes,
                                                     const int* __restrict__ tile_box, BatchPops<ST> in,
                                                     BatchPops<ST> out, const double* __restrict__ psi) {
  using H = typename BatchPops<ST>::Elem;
  KParams P;
#pragma unroll
  for (int k = 0; k < LBM_MAX_Q; ++k) P.mrt_c[k] = K.mrt_c[k];
  P.mrt_rows = K.mrt_rows;
#pragma unroll
  for (int d = 0; d < 3; ++d) P.accel[d] = K.accel[d];
  const TileRange tr = tile_range(K.ntiles);
  for (unsigned t = tr.t; t < tr.end; t += tr.stride) {
    const int bx = __builtin_amdgcn_readfirstlane(tile_box[t]);
    const BoxK& B = boxes[bx];
    const unsigned cell = (t - B.first_tile) * (unsigned)K.tile + threadIdx.x;
    if (cell >= B.cells) continue;
    const Coord c = box_coord(cell, B);
    const unsigned bits = B.walls ? K.bb[B.bb_off + cell] : 0u;
    P.cells = (int)B.cells;
    P.omega = B.omega;
#pragma unroll
    for (int s = 0; s < LBM_MAX_NC; ++s) P.gamma[s] = B.gamma[s];
    const int nc = B.nc;
    if (nc == 1) kbi_collide_cell<LAT, 1, H, COLL, FORC>(K, P, B, bx, in, out, c, cell, bits, psi);
    if constexpr (NCMAX >= 2)
      if (nc == 2) kbi_collide_cell<LAT, 2, H, COLL, FORC>(K, P, B, bx, in, out, c, cell, bits, psi);
    if constexpr (NCMAX >= 3)
      if (nc == 3) kbi_collide_cell<LAT, 3, H, COLL, FORC>(K, P, B, bx, in, out, c, cell, bits, psi);
    if constexpr (NCMAX >= 4)
      if (nc == 4) kbi_collide_cell<LAT, 4, H, COLL, FORC>(K, P, B, bx, in, out, c, cell, bits, psi);
  }
}

// ---------------------------------------------------------------------------
// Fused step (D2Q9, interleaved offsets): one launch per step instead of the psi
// pass and the collide pass.  A tile's cells are consecutive in the box's
// row-major order; the workgroup computes psi for them and their neighbours into
// LDS (its own cells from the pull it keeps for their collision, the others from a
// density-only pull) and collides after a barrier.  LDS holds padded rows of
// nx + 2 slots, x = -1 .. nx, the two ends being the periodic images of x = nx - 1
// and x = 0: with the padded index p(x, y) = y (nx + 2) + x + 1 of the unwrapped
// row-major order, slot s holds psi at p = base + s, base = p(t0) - (nx + 3), and
// every neighbour of a tile cell sits at the cell's own slot + c_y (nx + 2) + c_x
// (no wrap on the read side; the rows are wrapped in y where psi is computed).
// The slots span p(t0 + T - 1) - p(t0) + 2 (nx + 3) + 1 <= 3 T + 2 nx + 8.  Psi and
// the collision are kbi_psi_cell's and kbi_collide_cell's arithmetic, so the
// populations equal the two passes' bit for bit; the two-pass psi array is not
// written.
// ---------------------------------------------------------------------------

// psi of `cell` (kb_psi_ilv's arithmetic); f receives the cell's pull, zeros for a
// solid cell
template <int LAT, int NC, typename H>
__device__ __forceinline__ double kbi_psi_pull(const BatchK& K, const BoxK& B, int bx, const IlvBufs<H, NC, VS<LAT>::Q>& Bf,
                                               unsigned cell, float (&f)[NC][VS<LAT>::Q]) {
  constexpr int Q = VS<LAT>::Q;
  const unsigned bits = B.walls ? K.bb[B.bb_off + cell] : 0u;
  if (bits >> kSolidBit) {
#pragma unroll
    for (int s = 0; s < NC; ++s)
#pragma unroll
      for (int a = 0; a < Q; ++a) f[s][a] = 0.0f;
    return B.psi_wall;
  }
  ilv_pull_cell<LAT, NC, H, kbi_load_policy<H>()>(Bf, box_coord(cell, B), cell, bits, B.walls != 0, f);
  double rb[LBM_MAX_NC];
#pragma unroll
  for (int s = 0; s < LBM_MAX_NC; ++s) rb[s] = 0.0;
#pragma unroll
  for (int s = 0; s < NC; ++s) {
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < Q; ++a) acc += (double)f[s][a];
    rb[s] = acc;
  }
  return box_psi(K, B, bx, rb);
}

// bytes of LDS the fused step needs for tiles of `tile` cells and rows up to nx_max
inline size_t fused_lds_bytes(int tile, int nx_max) { return (size_t)(3 * tile + 2 * nx_max + 8) * sizeof(double); }

// one tile of the fused step; every thread of the workgroup calls it (two barriers)
template <int LAT, int NC, typename H, int COLL, int FORC>
__device__ __forceinline__ void kbi_fused_tile(const BatchK& K, const KParams& P, const BoxK& B, int bx,
                                               const BatchIlvPops<H>& in, const BatchIlvPops<H>& out, unsigned t0,
                                               double* sh) {
  using V = VS<LAT>;
  constexpr int Q = V::Q;
  const int T = K.tile, tid = (int)threadIdx.x;
  const int nx = B.nx, ny = B.ny, W = nx + 2;
  const unsigned cells = B.cells;
  const auto Bf = in.template bufs<NC, Q>(B);
  const auto pad = [nx, W](unsigned i) { return (int)(i / (unsigned)nx) * W + (int)(i % (unsigned)nx) + 1; };
  const int base = pad(t0) - (W + 1);
  const int span = pad(t0 + (unsigned)T - 1u) + (W + 1) - base + 1;
  // own cell (or, past the box's last cell, its periodic image), kept for the collision
  const unsigned lin = t0 + (unsigned)tid;
  const bool own = lin < cells;
  const int my = pad(lin) - base;
  float f[NC][Q];
  sh[my] = kbi_psi_pull<LAT, NC, H>(K, B, bx, Bf, own ? lin : lin % cells, f);
  // the other slots: neighbours outside the tile and the periodic images
  for (int s = tid; s < span; s += T) {
    const int p = base + s;
    const int y = p >= 0 ? p / W : -((W - 1 - p) / W);   // floor division
    const int xp = p - y * W - 1;                          // -1 .. nx
    const long long l = (long long)y * nx + xp;
    if (xp >= 0 && xp < nx && l >= (long long)t0 && l < (long long)t0 + T) continue;   // a tile thread's slot
    const int x = xp < 0 ? nx - 1 : (xp >= nx ? 0 : xp);
    const int yw = ((y % ny) + ny) % ny;
    float g[NC][Q];
    sh[s] = kbi_psi_pull<LAT, NC, H>(K, B, bx, Bf, (unsigned)(yw * nx + x), g);
  }
  __syncthreads();
  if (own) {
    double pn[Q];
#pragma unroll
    for (int a = 0; a < Q; ++a) pn[a] = sh[my + V::cy(a) * W + V::cx(a)];
    const unsigned bits = B.walls ? K.bb[B.bb_off + lin] : 0u;
    kbi_collide_pulled<LAT, NC, H, COLL, FORC>(K, P, B, bx, out, lin, !(bits >> kSolidBit), f, pn);
  }
  __syncthreads();   // the next tile overwrites sh
}

template <int LAT, int NCMAX, int ST, int COLL, int FORC>
__global__ __launch_bounds__(256) void kb_step_ilv(BatchK K, const BoxK* __restrict__ boxes,
                                                   const int* __restrict__ tile_box, BatchPops<ST> in,
                                                   BatchPops<ST> out) {
  static_assert(LAT == LBM_D2Q9 && ST != LBM_F64, "the fused step is built for D2Q9 offset storage");
  using H = typename BatchPops<ST>::Elem;
  extern __shared__ double sh_psi[];
  KParams P;
#pragma unroll
  for (int k = 0; k < LBM_MAX_Q; ++k) P.mrt_c[k] = K.mrt_c[k];
  P.mrt_rows = K.mrt_rows;
#pragma unroll
  for (int d = 0; d < 3; ++d) P.accel[d] = K.accel[d];
  const TileRange tr = tile_range(K.ntiles);
  for (unsigned t = tr.t; t < tr.end; t += tr.stride) {   // uniform per workgroup
    const int bx = __builtin_amdgcn_readfirstlane(tile_box[t]);
    const BoxK& B = boxes[bx];
    const unsigned t0 = (t - B.first_tile) * (unsigned)K.tile;
    P.cells = (int)B.cells;
    P.omega = B.omega;
#pragma unroll
    for (int s = 0; s < LBM_MAX_NC; ++s) P.gamma[s] = B.gamma[s];
    const int nc = B.nc;
    if (nc == 1) kbi_fused_tile<LAT, 1, H, COLL, FORC>(K, P, B, bx, in, out, t0, sh_psi);
    if constexpr (NCMAX >= 2)
      if (nc == 2) kbi_fused_tile<LAT, 2, H, COLL, FORC>(K, P, B, bx, in, out, t0, sh_psi);
    if constexpr (NCMAX >= 3)
      if (nc == 3) kbi_fused_tile<LAT, 3, H, COLL, FORC>(K, P, B, bx, in, out, t0, sh_psi);
    if constexpr (NCMAX >= 4)
      if (nc == 4) kbi_fused_tile<LAT, 4, H, COLL, FORC>(K, P, B, bx, in, out, t0, sh_psi);
  }
}

}  // namespace lbmk
