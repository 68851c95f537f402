// Device code of one time step (Sec. 3.4 order): population storage and decoding,
// the mixture EOS and psi (float64), the force stencil, the split and the
// per-component collision with forcing, plus the kernels built from them.
#pragma once
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <type_traits>

#include "lattice.hpp"
#include "lbm.h"

namespace lbmk {

constexpr int kBlock = 256;

// Per-run constants handed to every kernel by value.
struct KParams {
  int nx, ny, nz, cells;
  int plane_cells, nplanes;        // planes of the slowest axis (y in 2-D, z in 3-D)
  double RT;                       // R * T
  double G, beta, omega;           // omega = 1 / tau
  double aa[LBM_MAX_NC][LBM_MAX_NC];  // sqrt(a_i alpha_i a_j alpha_j)(1 - zeta_ij)
  double b[LBM_MAX_NC];
  double invM[LBM_MAX_NC];
  double gamma[LBM_MAX_NC];
  double mrt_c[LBM_MAX_Q];         // MRT: (1 - rate) / squared norm of each moment row
  unsigned mrt_rows;               // MRT: bit k set when mrt_c[k] != 0 (rows at rate 1 are skipped)
  double accel[3];
  int* err;                        // device error flag (set to 1 on a domain violation)
  // solid walls (null: none): per cell, bit a set when the source x - e_a of
  // direction a is solid (halfway bounce-back), bit 31 when the cell itself is solid
  const unsigned* bb = nullptr;
  double psi_wall = 0.0;           // psi of solid cells in the force stencil (wetting)
};
constexpr unsigned kSolidBit = 31u;

// Raw buffer access for the population planes: a scalar buffer descriptor per
// component, a per-lane byte offset in a vector register and a wavefront-uniform
// byte offset (direction plane, and in the row-structured kernels the row) in a
// scalar register.  Descriptor word 3 is the gfx9 raw-buffer format (32-bit data
// format, no swizzle, no index stride); num_records is the size of the
// component's planes.  Every offset is formed inside the planes by construction
// (cell and row indices below the box's cell count, planes below 4 GiB: host check).
using rsrc_t = __amdgpu_buffer_rsrc_t;
__device__ __forceinline__ rsrc_t make_rsrc(const void* p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
// CP: the instruction's cache-policy bits (bit 1 = nt, non-temporal: the line is
// not kept for reuse).  Each population plane is read once per pass (the psi pass
// and the collide pass read it once each) and written once per step, while the
// per-cell bases and psi are read again from the source rows of three planes; the
// population loads are therefore non-temporal, so that they do not evict the lines
// that are read again.  Stores keep the default policy (measured: non-temporal
// stores speed up the next psi pass but slow the collide pass by more).
constexpr int kPopLoad = 2;
constexpr int kPopStore = 0;
constexpr int kBaseStore = 0;
// 1.0f that the compiler cannot fold (an empty asm statement owns its value, no
// instruction is emitted).  w + r with r widened from float16 is then written
// fmaf(r, one, w): r * 1 is exact, so the result is the float32 sum itself, and it
// compiles to one mixed-precision FMA (v_fma_mix_f32 reading r as float16) in
// place of a conversion and an add.
__device__ __forceinline__ float opaque_one() {
  float one = 1.0f;
  asm("" : "+s"(one));
  return one;
}
// w + r (float32 sum) for an offset r loaded as float16 (or float32)
__device__ __forceinline__ float w_plus(float w, float r, float one) { return __builtin_fmaf(r, one, w); }

template <int CP = 0>
__device__ __forceinline__ double bload(rsrc_t r, unsigned voff, unsigned soff, double) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, CP));
}
template <int CP = 0>
__device__ __forceinline__ float bload(rsrc_t r, unsigned voff, unsigned soff, float) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, CP));
}
template <int CP = 0>
__device__ __forceinline__ float bload(rsrc_t r, unsigned voff, unsigned soff, __half) {
  return __half2float(__builtin_bit_cast(__half, __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, CP)));
}
template <int CP = 0>
__device__ __forceinline__ void bstore(rsrc_t r, unsigned voff, unsigned soff, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0)), v),
                                        r, voff, soff, CP);
}
template <int CP = 0>
__device__ __forceinline__ void bstore(rsrc_t r, unsigned voff, unsigned soff, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, CP);
}
template <int CP = 0>
__device__ __forceinline__ void bstore(rsrc_t r, unsigned voff, unsigned soff, __half v) {
  __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, voff, soff, CP);
}

// ---------------------------------------------------------------------------
// Population storage.  float64: planes [nc][Q][cells], the stored value of
// direction a at cell y being the post-collision population that streams to
// y + e_a.  The offset formats (IlvPops below) store base(y) (w_a + r_a(y)) with
// the components of a cell side by side.  comp(s) returns a view of component s;
// get(a, idx) decodes direction a at cell idx, put_all stores the Q
// post-collision values (and, for the offset formats, the base) of a cell.  The
// offset formats rescale the stored base after rounding the offsets so that the
// cell's decoded mass equals its mass before encoding (encode_offsets); the
// caller passes that mass summed in float64.
// ---------------------------------------------------------------------------
template <int ST>
struct Pops;

template <>
struct Pops<LBM_F64> {
  using R = double;   // collision arithmetic
  double* f;
  struct View {
    rsrc_t rf;
    unsigned plane;   // bytes per direction plane
    __device__ __forceinline__ double get(int a, unsigned idx, double) const {
      return bload<kPopLoad>(rf, idx * 8u, (unsigned)a * plane, 0.0);
    }
    // per-lane direction plane: pbytes = direction * plane
    __device__ __forceinline__ double get_at(unsigned idx, unsigned pbytes, double) const {
      return bload<kPopLoad>(rf, idx * 8u + pbytes, 0u, 0.0);
    }
    // all Q directions, direction a from cell src(a): loads first, then decode
    template <int Q, typename Src, typename W>
    __device__ __forceinline__ void get_all(Src src, double* out, W) const {
#pragma unroll
      for (int a = 0; a < Q; ++a) out[a] = bload<kPopLoad>(rf, src(a) * 8u, (unsigned)a * plane, 0.0);
    }
    template <int Q, typename W>
    __device__ __forceinline__ void put_all(unsigned idx, const double* v, double, W) const {
#pragma unroll
      for (int a = 0; a < Q; ++a) bstore<kPopStore>(rf, idx * 8u, (unsigned)a * plane, v[a]);
    }
    // row-structured forms: per-lane offset xo within the row, wave-uniform row
    // offset ro (in cells) folded into the scalar offset of the buffer instruction
    __device__ __forceinline__ double get_row(int a, unsigned xo, unsigned ro, double) const {
      return bload<kPopLoad>(rf, xo * 8u, (unsigned)a * plane + ro * 8u, 0.0);
    }
    template <int Q, bool MIX = false, typename W>
    __device__ __forceinline__ void put_all_row(unsigned xo, unsigned ro, const double* v, double, W) const {
#pragma unroll
      for (int a = 0; a < Q; ++a) bstore<kPopStore>(rf, xo * 8u, (unsigned)a * plane + ro * 8u, v[a]);
    }
  };
  __device__ __forceinline__ View comp(int s, int Q, int cells) const {
    const unsigned plane = (unsigned)cells * 8u;
    return View{make_rsrc(f + (size_t)s * Q * cells, (unsigned)Q * plane), plane};
  }
};

// n / d for d in [1/2, 2] (float64): hardware reciprocal, one Newton step on it
// and one residual correction of the quotient -- far below the float32 rounding
// the result goes through
__device__ __forceinline__ double div_refined(double n, double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(fma(-d, r, 1.0), r, r);
  const double q = n * r;
  return fma(fma(-d, q, n), r, q);
}

// float32 -> storage type of an offset (float16: round to nearest even)
template <typename H>
__device__ __forceinline__ H enc_offset(float v) {
  if constexpr (std::is_same<H, __half>::value) return __float2half_rn(v);
  else return v;
}

// Offset encoding of the Q post-collision values v of one cell and component.
// v: the values; mass: the cell's mass of this component (sum of v, summed exactly
// in float64); w(a): weights.  Writes the offsets r[a] and returns the base to store.
// The offsets are taken against b0 = +-sum_a |v_a| with the sign of the mass,
// which is the mass wherever every population has the sign of the mass (a
// positive cell, or a trace component whose density is negative throughout
// the cell): the offsets then hold only the small non-equilibrium part.  Where
// the populations change sign (a density near zero) |b0| stays of the size of
// the populations, so the offsets stay bounded and their rounding stays
// relative to the populations themselves.  After rounding the offsets the stored
// base is mass / S with S = sum_a (w_a + r_a), each term formed in float32
// exactly as the decoder forms it and the sum taken in float64 (exact); a cell
// at rest is then a fixed point of encode/stream/decode, since the decoder's
// product roundings total less than half an ulp of the base, which the
// rounding of mass / S absorbs.  Float32 sums instead bias the mass by a
// fraction of an ulp per step, coherently over a bulk phase, which over
// thousands of steps shifts phase compositions by ~1e-4.  Where the
// populations are far from one sign (S < 1/2) the base stays b0.
// MIX: form w + r with the mixed-precision FMA (the same float32 value).
template <int Q, typename H, bool MIX, typename W>
__device__ __forceinline__ float encode_offsets(const float* v, double mass, W w, H* r) {
  float b0 = 0.0f;
#pragma unroll
  for (int a = 0; a < Q; ++a) b0 += fabsf(v[a]);
  if (mass < 0.0) b0 = -b0;
  // hardware reciprocal (1 ulp): its error is absorbed by the rescaled base
  const float inv = (b0 != 0.0f) ? __builtin_amdgcn_rcpf(b0) : 0.0f;
  const float wm = (b0 != 0.0f) ? 1.0f : 0.0f;
  double S = 0.0;
  const float one = opaque_one();
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    r[a] = enc_offset<H>(v[a] * inv - wm * w(a));
    if constexpr (MIX) S += (double)w_plus(w(a), (float)r[a], one);
    else S += (double)(w(a) + (float)r[a]);
  }
  return S >= 0.5 ? (float)div_refined(mass, S) : b0;
}

// Component-interleaved offsets: the offsets of every component of one direction
// and cell sit together, r[(a cells + y) nc + s], and so do the bases,
// base[y nc + s]; one vector access moves all nc components of a cell (the step
// kernels k_psi_ilv / k_collide_ilv, and kb_psi_ilv / kb_collide_ilv per box).
// comp(s) views component s with strided scalar accesses, for the kernels around
// the step (moments, export, import, the adjoint).  Decoding: f_a = b (w_a + r_a).
template <typename H>
struct IlvPops {
  using R = float;
  using Elem = H;
  float* base;
  H* r;
  int nc;
  struct View {
    rsrc_t rb, rr;
    unsigned plane;   // bytes per direction plane of r (cells nc sizeof(H))
    unsigned rs, ro;  // bytes between cells in r; byte offset of this component
    unsigned bs, bo;  // the same for the base
    using Elem = H;
    __device__ __forceinline__ float get(int a, unsigned idx, float w) const {
      return bload(rb, idx * bs + bo, 0u, 0.0f) * (w + bload<kPopLoad>(rr, idx * rs + ro, (unsigned)a * plane, H()));
    }
    __device__ __forceinline__ float get_at(unsigned idx, unsigned pbytes, float w) const {
      return bload(rb, idx * bs + bo, 0u, 0.0f) * (w + bload<kPopLoad>(rr, idx * rs + ro + pbytes, 0u, H()));
    }
    template <int Q, typename W>
    __device__ __forceinline__ void put_all(unsigned idx, const float* v, double mass, W w) const {
      H rq[Q];
      const float b = encode_offsets<Q, H, false>(v, mass, w, rq);
#pragma unroll
      for (int a = 0; a < Q; ++a) bstore<kPopStore>(rr, idx * rs + ro, (unsigned)a * plane, rq[a]);
      bstore<kBaseStore>(rb, idx * bs + bo, 0u, b);
    }
  };
  __device__ __forceinline__ View comp(int s, int Q, int cells) const {
    const unsigned cs = (unsigned)nc * (unsigned)sizeof(H);
    const unsigned plane = (unsigned)cells * cs;
    return View{make_rsrc(base, (unsigned)cells * (unsigned)nc * 4u), make_rsrc(r, (unsigned)Q * plane), plane, cs,
                (unsigned)s * (unsigned)sizeof(H), (unsigned)nc * 4u, (unsigned)s * 4u};
  }
};

template <>
struct Pops<LBM_F32_OFS> : IlvPops<float> {};
template <>
struct Pops<LBM_F16_OFS> : IlvPops<__half> {};

// Cell coordinates with periodic neighbours; at(dx,dy,dz) is the linear index of
// the neighbour at offset (dx, dy, dz).
struct Coord {
  unsigned xs[3], ys[3], zs[3];   // [x-1, x, x+1], row offsets, plane offsets
  __device__ __forceinline__ unsigned at(int dx, int dy, int dz) const {
    return zs[dz + 1] + ys[dy + 1] + xs[dx + 1];
  }
};

__device__ __forceinline__ Coord make_coord(unsigned cell, const KParams& P) {
  const unsigned nx = P.nx, ny = P.ny, nz = P.nz;
  const unsigned x = cell % nx;
  const unsigned t = cell / nx;
  const unsigned y = t % ny;
  const unsigned z = t / ny;
  Coord c;
  c.xs[0] = x == 0 ? nx - 1 : x - 1;
  c.xs[1] = x;
  c.xs[2] = x == nx - 1 ? 0 : x + 1;
  c.ys[0] = (y == 0 ? ny - 1 : y - 1) * nx;
  c.ys[1] = y * nx;
  c.ys[2] = (y == ny - 1 ? 0 : y + 1) * nx;
  const unsigned pl = nx * ny;
  c.zs[0] = (z == 0 ? nz - 1 : z - 1) * pl;
  c.zs[1] = z * pl;
  c.zs[2] = (z == nz - 1 ? 0 : z + 1) * pl;
  return c;
}

// Row-structured position: a wavefront covers 64 consecutive x of one row (y, z),
// so the row part of every neighbour offset is uniform across the wavefront
// (scalar registers, passed as the buffer instructions' scalar offset) and only
// x - 1, x, x + 1 (periodic) live in vector registers.
struct RowCoord {
  unsigned xs[3];          // per lane: x-1, x, x+1
  unsigned ys[3], zs[3];   // uniform: (y+dy) nx and (z+dz) nx ny, dy, dz in -1..1
  unsigned x0;             // uniform: x of lane 0
  __device__ __forceinline__ unsigned row(int dy, int dz) const { return zs[dz + 1] + ys[dy + 1]; }
  __device__ __forceinline__ unsigned x(int dx) const { return xs[dx + 1]; }
};

// Segment `seg` of the launch (uniform): rows of planes [plane0, plane0 + nplanes)
// (periodic), each row cut into ceil(nx / 64) segments of 64 cells.  False when
// the segment lies past the range; *in_row is false for lanes with x >= nx.
template <int D>
__device__ __forceinline__ bool row_segment(const KParams& P, unsigned seg, int plane0, int nplanes, unsigned lane,
                                            RowCoord* c, bool* in_row) {
  const unsigned nx = P.nx, ny = P.ny, nz = P.nz;
  const unsigned nseg = (nx + 63u) / 64u;
  const unsigned rows_pp = D == 3 ? ny : 1u;
  if (seg >= (unsigned)nplanes * rows_pp * nseg) return false;
  const unsigned sx = seg % nseg, r = seg / nseg;
  unsigned y, z;
  if (D == 3) {
    y = r % ny;
    z = (unsigned)plane0 + r / ny;
    if (z >= nz) z -= nz;
  } else {
    y = (unsigned)plane0 + r;
    if (y >= ny) y -= ny;
    z = 0;
  }
  c->x0 = sx * 64u;
  const unsigned x = c->x0 + lane;
  *in_row = x < nx;
  const unsigned xx = *in_row ? x : 0u;
  c->xs[0] = xx == 0 ? nx - 1 : xx - 1;
  c->xs[1] = xx;
  c->xs[2] = xx == nx - 1 ? 0 : xx + 1;
  c->ys[0] = (y == 0 ? ny - 1 : y - 1) * nx;
  c->ys[1] = y * nx;
  c->ys[2] = (y == ny - 1 ? 0 : y + 1) * nx;
  const unsigned pl = nx * ny;
  c->zs[0] = (z == 0 ? nz - 1 : z - 1) * pl;
  c->zs[1] = z * pl;
  c->zs[2] = (z == nz - 1 ? 0 : z + 1) * pl;
  return true;
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2).
// Launches use a multiple of 8 workgroups and remap workgroup b to the logical
// block (b mod 8) * (n / 8) + b / 8, so each XCD sweeps one contiguous range of
// cells and the cache lines shared by neighbouring blocks stay in one L2.
constexpr unsigned kXcd = 8;
__device__ __forceinline__ unsigned logical_block() {
  const unsigned n = gridDim.x, b = blockIdx.x;
  return (b % kXcd) * (n / kXcd) + b / kXcd;
}
inline unsigned xcd_grid(unsigned blocks) { return (blocks + kXcd - 1) / kXcd * kXcd; }

// Linear index of the k-th cell of a launch covering `nplanes` planes starting at
// plane `plane0` (periodic in the plane index); false past the end.
template <int B = kBlock>   // B: threads per workgroup of the launch
__device__ __forceinline__ bool launch_cell(const KParams& P, int plane0, int nplanes, unsigned* cell) {
  const unsigned lin = logical_block() * B + threadIdx.x;
  const unsigned pc = P.plane_cells;
  if (lin >= (unsigned)nplanes * pc) return false;
  const unsigned k = lin / pc;
  unsigned plane = plane0 + k;
  if (plane >= (unsigned)P.nplanes) plane -= P.nplanes;
  *cell = plane * pc + (lin - k * pc);
  return true;
}

__device__ __forceinline__ void flag_error(const KParams& P) { *P.err = 1; }

// Mixture Peng-Robinson pressure from cell-volume densities (Eq. MCPengRobinson with
// the random mixing rule written in molar densities n_i = rbar_i / M_i:
// b_m rho~ = sum b_i n_i, [a alpha]_m rho~^2 = sum_ij n_i n_j (a alpha)_ij).
template <int NC>
__device__ __forceinline__ double eos_pressure(const KParams& P, const double* rb, double* Bn_out) {
  double n[NC];
  double rt = 0.0, Bn = 0.0;
#pragma unroll
  for (int i = 0; i < NC; ++i) {
    n[i] = rb[i] * P.invM[i];
    rt += n[i];
    Bn += P.b[i] * n[i];
  }
  double An = 0.0;
#pragma unroll
  for (int i = 0; i < NC; ++i) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < NC; ++j) s += P.aa[i][j] * n[j];
    An += n[i] * s;
  }
  *Bn_out = Bn;
  return rt * P.RT / (1.0 - Bn) - An / (1.0 + 2.0 * Bn - Bn * Bn);
}

// psi = sqrt(2 (p_EOS - c_s^2 rho) / (G c_s^2)), Eq. (psicorrected), dt = 1.
template <int NC>
__device__ __forceinline__ double eos_psi(const KParams& P, const double* rb) {
  double Bn;
  const double p = eos_pressure<NC>(P, rb, &Bn);
  double rho = 0.0;
#pragma unroll
  for (int i = 0; i < NC; ++i) rho += rb[i];
  const double X = 6.0 * (p - rho * (1.0 / 3.0)) / P.G;
  if (!(Bn < 1.0) || !(X >= 0.0) || !(X <= 1.0e300)) flag_error(P);
  return sqrt(X);
}

// Density of component s at the cell and its momentum contribution, summed in the
// collision precision R (float64 for float64 storage; float32 for the offset
// formats, whose decoded populations carry float32 precision), returned as float64.
// Population of direction a arriving at cell `own` with walls: streamed from the
// neighbour nbr = own - e_a, or, when bit a of the cell's wall mask is set (nbr is
// solid), the cell's own post-collision population of the opposite direction
// (halfway bounce-back; w_a equals the opposite direction's weight).
template <int LAT, typename View, typename R>
__device__ __forceinline__ R pull_bb(const View& cv, int a, unsigned bits, unsigned own, unsigned nbr, R w) {
  const bool back = (bits >> a) & 1u;
  return cv.get_at(back ? own : nbr, (unsigned)(back ? VS<LAT>::opp(a) : a) * cv.plane, w);
}

template <int LAT, int ST>
__device__ __forceinline__ double pull_moments(const KParams& P, const Pops<ST>& in, int s, const Coord& c,
                                               typename Pops<ST>::R* j, unsigned cell = 0, unsigned bits = 0) {
  using V = VS<LAT>;
  using R = typename Pops<ST>::R;
  const auto cv = in.comp(s, V::Q, P.cells);
  R acc = 0;
  R jx = 0, jy = 0, jz = 0;
#pragma unroll
  for (int a = 0; a < V::Q; ++a) {
    const unsigned nbr = c.at(-V::cx(a), -V::cy(a), -V::cz(a));
    const R v = P.bb ? pull_bb<LAT>(cv, a, bits, cell, nbr, (R)V::w(a)) : cv.get(a, nbr, (R)V::w(a));
    acc += v;
    if (V::cx(a)) jx += (R)V::cx(a) * v;
    if (V::cy(a)) jy += (R)V::cy(a) * v;
    if (V::cz(a)) jz += (R)V::cz(a) * v;
  }
  j[0] += jx;
  j[1] += jy;
  j[2] += jz;
  return (double)acc;
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

// a / b in the collision precision: float64 divides (correctly rounded); float32
// multiplies by the hardware reciprocal (1 ulp), an error below the float32
// collision's own rounding, in place of the ~10-instruction exact division.
__device__ __forceinline__ double quot(double a, double b) { return a / b; }
__device__ __forceinline__ float quot(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }

// Compile-time loop: f(integral_constant<int, I>) for I in [B, E).
template <int B, int E, typename Fn>
__device__ __forceinline__ void static_for(Fn&& fn) {
  if constexpr (B < E) {
    fn(std::integral_constant<int, B>{});
    static_for<B + 1, E>(fn);
  }
}

// Equilibrium of Eq. (equilibrium a) for direction a.
template <int LAT, typename R>
__device__ __forceinline__ R feq(int a, R rho, R ux, R uy, R uz, R uu) {
  using V = VS<LAT>;
  const R eu = (R)V::cx(a) * ux + (R)V::cy(a) * uy + (R)V::cz(a) * uz;
  return rho * (R)V::w(a) * ((R)1 + (R)3 * eu + (R)4.5 * eu * eu - (R)1.5 * uu);
}

// Collision with forcing of one component followed by the store of its Q
// post-collision populations at `cell` (pull streaming: the next step reads
// direction a of this cell from the neighbour at cell + e_a).
//   f   : populations of component s at this cell (time t, post-streaming)
//   rs  : rbar_s;  u: equilibrium velocity (Guo: the shared (j + F_total/2)/rho;
//         EDM: that velocity minus du_s/2, per component);  Fs: F_s (Guo) or du_s (EDM)
// BGK : f* = f - omega (f - feq) + (1 - omega/2) S_guo        | + [feq(u + du) - feq(u)]
// MRT : f* = f + src - M^-1 S M (f - feq + h src), h = 1/2 (Guo), 0 (EDM), which
//       with d = f - feq + h src is the same as
//       f* = feq + (1 - h) src + M^-1 (I - S) M d
//       (M^-1 = M^T diag(1/|M_k|^2) for the orthogonal basis; with EDM, h = 0 and
//       feq + src = feq(u + du), which is evaluated as such).  Rows relaxed at
//       rate 1 drop out of the second form, so only the rows with rate != 1 are
//       transformed (a uniform branch per row; the density row always drops out
//       because sum_a d_a = 0).
// Everything is evaluated on opposite pairs (a, opp(a)): the equilibrium and the
// sources split into a part even under e -> -e and an odd part,
//   feq_a = E + O, feq_opp = E - O,  E = w rs (1 + 9/2 (e.u)^2 - 3/2 u.u), O = 3 w rs e.u,
//   Guo : w[3(e - u).F + 9 (e.u)(e.F)]  -> even w(9 (e.u)(e.F) - 3 u.F), odd 3 w e.F,
//   EDM : feq(u + du) - feq(u) = w rs [3 e.du + 9/2 (e.du)(2 e.u + e.du) - 3/2 du.(2u + du)]
//         -> even w rs (9/2 (e.du)(2 e.u + e.du) - 3/2 du.(2u + du)), odd 3 w rs e.du;
// MRT even rows act on d_a + d_opp, odd rows on d_a - d_opp.  With EDM the rows
// take the raw pair sums of f and subtract the equilibrium's moments, quadratic in
// u with compile-time coefficients (feq(u) is never formed per velocity); rows
// whose entries depend on |e_a|^2 alone (e, epsilon) are taken on the speed-class
// sums and relaxed back onto the classes.
template <int LAT, typename R, int COLL, int FORC, typename Sink>
__device__ __forceinline__ void collide_values(const KParams& P, const R* f, R rs, const R* u3, const R* F3,
                                               Sink sink) {
  using V = VS<LAT>;
  constexpr int Q = V::Q;
  constexpr int NP = (Q - 1) / 2;
  const R ux = u3[0], uy = u3[1], uz = u3[2];
  const R uu = ux * ux + uy * uy + uz * uz;
  const R Fx = F3[0], Fy = F3[1], Fz = F3[2];
  const R uF = ux * Fx + uy * Fy + uz * Fz;                       // Guo: u.F_s
  const R dvv = Fx * ((R)2 * ux + Fx) + Fy * ((R)2 * uy + Fy) + Fz * ((R)2 * uz + Fz);  // EDM: du.(2u+du)
  const R base1 = (R)1 - (R)1.5 * uu;
  // even / odd parts of feq and of the source for velocity a (a > 0) or the rest (a = 0)
  auto parts = [&](auto A, R& Ev, R& Od, R& sE, R& sO) {
    constexpr int a = decltype(A)::value;
    constexpr R cx = V::cx(a), cy = V::cy(a), cz = V::cz(a);
    const R wr = (R)V::w(a) * rs;
    const R eu = cx * ux + cy * uy + cz * uz;
    Ev = wr * (base1 + (R)4.5 * eu * eu);
    Od = (R)3 * wr * eu;
    if constexpr (FORC == LBM_GUO) {
      const R eF = cx * Fx + cy * Fy + cz * Fz;
      sE = (R)V::w(a) * ((R)9 * eu * eF - (R)3 * uF);
      sO = (R)3 * (R)V::w(a) * eF;
    } else {
      const R ed = cx * Fx + cy * Fy + cz * Fz;
      sE = wr * ((R)4.5 * ed * ((R)2 * eu + ed) - (R)1.5 * dvv);
      sO = (R)3 * wr * ed;
    }
  };
  R fo[Q];
  if constexpr (COLL == LBM_BGK) {
    const R om = (R)P.omega;
    const R gpre = (FORC == LBM_GUO) ? (R)1 - (R)0.5 * om : (R)1;
    {
      R Ev, Od, sE, sO;
      parts(std::integral_constant<int, 0>{}, Ev, Od, sE, sO);
      fo[0] = f[0] - om * (f[0] - Ev) + gpre * sE;
    }
    static_for<0, NP>([&](auto Pp) {
      constexpr int p = decltype(Pp)::value;
      constexpr int a = V::pair_first(p), b = V::opp(V::pair_first(p));
      R Ev, Od, sE, sO;
      parts(std::integral_constant<int, a>{}, Ev, Od, sE, sO);
      fo[a] = f[a] - om * (f[a] - (Ev + Od)) + gpre * (sE + sO);
      fo[b] = f[b] - om * (f[b] - (Ev - Od)) + gpre * (sE - sO);
    });
  } else {
    // Z0, ZE[p], ZO[p]: rest, even and odd pair values whose row projections, plus
    // moff(k), are the moments of the deviation d; X0, XE[p], XO[p]: the state the
    // relaxed deviations are added to (feq + (1 - h) src)
    R Z0, X0, ZE[NP], ZO[NP], XE[NP], XO[NP];
    if constexpr (FORC == LBM_EDM) {
      // h = 0, d = f - feq(u): only d's moments enter, the raw moments of f minus
      // those of feq(u) (moff); feq(u) + [feq(u + du) - feq(u)] = feq(u + du) is
      // formed directly
      const R vx = ux + Fx, vy = uy + Fy, vz = uz + Fz;
      const R basev = (R)1 - (R)1.5 * (vx * vx + vy * vy + vz * vz);
      Z0 = f[0];
      X0 = (R)V::w(0) * rs * basev;
      static_for<0, NP>([&](auto Pp) {
        constexpr int p = decltype(Pp)::value;
        constexpr int a = V::pair_first(p), b = V::opp(V::pair_first(p));
        constexpr R cx = V::cx(a), cy = V::cy(a), cz = V::cz(a);
        const R wr = (R)V::w(a) * rs;
        const R ev = cx * vx + cy * vy + cz * vz;
        ZE[p] = f[a] + f[b];
        ZO[p] = f[a] - f[b];
        XE[p] = wr * (basev + (R)4.5 * ev * ev);
        XO[p] = (R)3 * wr * ev;
      });
    } else {
      const R h = (R)0.5, g1 = (R)0.5;
      R Ev, Od, sE, sO;
      parts(std::integral_constant<int, 0>{}, Ev, Od, sE, sO);
      Z0 = f[0] - Ev + h * sE;
      X0 = Ev + g1 * sE;
      static_for<0, NP>([&](auto Pp) {
        constexpr int p = decltype(Pp)::value;
        constexpr int a = V::pair_first(p), b = V::opp(V::pair_first(p));
        R Ev, Od, sE, sO;
        parts(std::integral_constant<int, a>{}, Ev, Od, sE, sO);
        ZE[p] = (f[a] + f[b]) - (R)2 * Ev + (R)2 * h * sE;   // d_a + d_b
        ZO[p] = (f[a] - f[b]) - (R)2 * Od + (R)2 * h * sO;   // d_a - d_b
        XE[p] = Ev + g1 * sE;                               // feq + (1 - h) src
        XO[p] = Od + g1 * sO;
      });
    }
    // EDM: minus row k's moment of feq(u), rs times a quadratic in u (eq_c0/1/2)
    auto moff = [&](auto K) -> R {
      constexpr int k = decltype(K)::value;
      if constexpr (FORC == LBM_EDM) {
        const R uv[3] = {ux, uy, uz};
        R m = (R)eq_c0<LAT>(k);
        static_for<0, V::D>([&](auto I) {
          constexpr int ii = decltype(I)::value;
          if constexpr (eq_c1<LAT>(k, ii) != 0.0) m += (R)eq_c1<LAT>(k, ii) * uv[ii];
          static_for<ii, V::D>([&](auto J) {
            constexpr int jj = decltype(J)::value;
            constexpr double c2 = eq_c2<LAT>(k, ii, jj);
            if constexpr (c2 > 1e-12 || c2 < -1e-12) m += (R)c2 * (uv[ii] * uv[jj]);
          });
        });
        return -rs * m;
      } else {
        return (R)0;
      }
    };
    // skip rows relaxed at rate 1 (a uniform branch on a scalar bit mask); in
    // float64 the kernel streams at HBM speed and the branches cost more than the
    // skipped rows
    auto active = [&](int k) { return std::is_same<R, double>::value || ((P.mrt_rows >> k) & 1u); };
    // isotropic even rows (e, epsilon): projections of the speed-class sums of ZE,
    // relaxed onto the classes (the first contributions to the accumulators)
    R Zc1 = 0, Zc2 = 0;
    static_for<0, NP>([&](auto Pp) {
      constexpr int p = decltype(Pp)::value;
      if constexpr (speed2<LAT>(V::pair_first(p)) == 1) Zc1 += ZE[p];
      else Zc2 += ZE[p];
    });
    R acc0 = 0, inc1 = 0, inc2 = 0;
    static_for<1, Q>([&](auto K) {
      constexpr int k = decltype(K)::value;
      if constexpr (row_isotropic<LAT>(k) && !row_odd<LAT>(k)) {
        if (active(k)) {
          constexpr double c0 = mrow_class<LAT>(k, 0), c1 = mrow_class<LAT>(k, 1), c2 = mrow_class<LAT>(k, 2);
          R m = moff(K);
          if constexpr (c0 != 0.0) m += (R)c0 * Z0;
          if constexpr (c1 != 0.0) m += (R)c1 * Zc1;
          if constexpr (c2 != 0.0) m += (R)c2 * Zc2;
          m *= (R)P.mrt_c[k];
          if constexpr (c0 != 0.0) acc0 += (R)c0 * m;
          if constexpr (c1 != 0.0) inc1 += (R)c1 * m;
          if constexpr (c2 != 0.0) inc2 += (R)c2 * m;
        }
      }
    });
    R accE[NP], accO[NP];
    static_for<0, NP>([&](auto Pp) {
      constexpr int p = decltype(Pp)::value;
      accE[p] = speed2<LAT>(V::pair_first(p)) == 1 ? inc1 : inc2;
      accO[p] = 0;
    });
    // the other rows, one at a time: m = (row . Z + moff) c_k, back-projected
    static_for<1, Q>([&](auto K) {
      constexpr int k = decltype(K)::value;
      if constexpr (!(row_isotropic<LAT>(k) && !row_odd<LAT>(k))) {
        if (active(k)) {
          R m = moff(K);
          if constexpr (!row_odd<LAT>(k)) {
            if constexpr (V::mrow(k, 0) != 0.0) m += (R)V::mrow(k, 0) * Z0;
            static_for<0, NP>([&](auto Pp) {
              constexpr int p = decltype(Pp)::value;
              constexpr double mk = V::mrow(k, V::pair_first(p));
              if constexpr (mk != 0.0) m += (R)mk * ZE[p];
            });
          } else {
            static_for<0, NP>([&](auto Pp) {
              constexpr int p = decltype(Pp)::value;
              constexpr double mk = V::mrow(k, V::pair_first(p));
              if constexpr (mk != 0.0) m += (R)mk * ZO[p];
            });
          }
          m *= (R)P.mrt_c[k];
          if constexpr (!row_odd<LAT>(k) && V::mrow(k, 0) != 0.0) acc0 += (R)V::mrow(k, 0) * m;
          static_for<0, NP>([&](auto Pp) {
            constexpr int p = decltype(Pp)::value;
            constexpr double mk = V::mrow(k, V::pair_first(p));
            if constexpr (mk != 0.0) {
              if constexpr (row_odd<LAT>(k)) accO[p] += (R)mk * m;
              else accE[p] += (R)mk * m;
            }
          });
        }
      }
    });
    fo[0] = X0 + acc0;
    static_for<0, NP>([&](auto Pp) {
      constexpr int p = decltype(Pp)::value;
      constexpr int a = V::pair_first(p), b = V::opp(V::pair_first(p));
      const R e = XE[p] + accE[p], o = XO[p] + accO[p];
      fo[a] = e + o;
      fo[b] = e - o;
    });
  }
  sink(fo);
}

// Equilibrium velocity and forcing input of component s at a cell, in the
// collision precision R (float64 for float64 storage, float32 otherwise):
//   Guo: u = (j + F_total/2)/rho (shared), F_s = chi_s F + rbar_s g;
//   EDM: u_s = (j + F_total/2)/rho - du_s/2, du_s = gamma_s F / Gamma + g (= F_s / rbar_s),
//        so that component s gains exactly F_s where it rests (Sec. 3.1,
//        Eq. hydrostatic1), as with Guo's term;
// chi_s = gamma_s rbar_s / Gamma, Gamma = sum gamma_i rbar_i (Eq. distributionforce).
template <int FORC, typename R>
__device__ __forceinline__ void cell_velocity_split(const KParams& P, int s, double rho, double Gam, const double* j,
                                                    const double* F, R rs, R* u, R* fs) {
  const R g0 = (R)P.accel[0], g1 = (R)P.accel[1], g2 = (R)P.accel[2];
  const R rhoR = (R)rho, irho = quot((R)1, rhoR);
  const R FR[3] = {(R)F[0], (R)F[1], (R)F[2]};
  const R ch = quot((R)P.gamma[s], (R)Gam);   // chi_s / rbar_s
  if (FORC == LBM_GUO) {
    // u = (j + F_total/2) / rho, F_total = F + rho g
    u[0] = ((R)j[0] + (R)0.5 * (FR[0] + rhoR * g0)) * irho;
    u[1] = ((R)j[1] + (R)0.5 * (FR[1] + rhoR * g1)) * irho;
    u[2] = ((R)j[2] + (R)0.5 * (FR[2] + rhoR * g2)) * irho;
    fs[0] = ch * rs * FR[0] + rs * g0;
    fs[1] = ch * rs * FR[1] + rs * g1;
    fs[2] = ch * rs * FR[2] + rs * g2;
  } else {
    // (j + F/2) / rho - (gamma_s / Gamma) F / 2: the g of F_total and of du_s cancel
    u[0] = ((R)j[0] + (R)0.5 * FR[0]) * irho - (R)0.5 * (ch * FR[0]);
    u[1] = ((R)j[1] + (R)0.5 * FR[1]) * irho - (R)0.5 * (ch * FR[1]);
    u[2] = ((R)j[2] + (R)0.5 * FR[2]) * irho - (R)0.5 * (ch * FR[2]);
    fs[0] = ch * FR[0] + g0;
    fs[1] = ch * FR[1] + g1;
    fs[2] = ch * FR[2] + g2;
  }
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

// Wavefront lane shifts (DPP wave_shr:1 / wave_shl:1): lane i takes lane i - 1
// (resp. i + 1); lane 0 (resp. 63), which has no source lane, keeps `fill`.
// Every lane of the wavefront must be active.
__device__ __forceinline__ float lane_from_left(float v, float fill) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, fill),
                                                               __builtin_bit_cast(int, v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float lane_from_right(float v, float fill) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, fill),
                                                               __builtin_bit_cast(int, v), 0x130, 0xf, 0xf, false));
}

__device__ __forceinline__ double lane_from_left(double v, double fill) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned long long g = __builtin_bit_cast(unsigned long long, fill);
  const float lo = lane_from_left(__builtin_bit_cast(float, (unsigned)u), __builtin_bit_cast(float, (unsigned)g));
  const float hi = lane_from_left(__builtin_bit_cast(float, (unsigned)(u >> 32)),
                                  __builtin_bit_cast(float, (unsigned)(g >> 32)));
  return __builtin_bit_cast(double, (unsigned long long)__builtin_bit_cast(unsigned, lo) |
                                        ((unsigned long long)__builtin_bit_cast(unsigned, hi) << 32));
}
__device__ __forceinline__ double lane_from_right(double v, double fill) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned long long g = __builtin_bit_cast(unsigned long long, fill);
  const float lo = lane_from_right(__builtin_bit_cast(float, (unsigned)u), __builtin_bit_cast(float, (unsigned)g));
  const float hi = lane_from_right(__builtin_bit_cast(float, (unsigned)(u >> 32)),
                                   __builtin_bit_cast(float, (unsigned)(g >> 32)));
  return __builtin_bit_cast(double, (unsigned long long)__builtin_bit_cast(unsigned, lo) |
                                        ((unsigned long long)__builtin_bit_cast(unsigned, hi) << 32));
}

// Source rows of a pull: (dy, dz) = (-c_y, -c_z) as index (dy + 1) + 3 (dz + 1).
template <int LAT>
__host__ __device__ constexpr int pull_row(int a) {
  return (1 - VS<LAT>::cy(a)) + 3 * (1 - VS<LAT>::cz(a));
}
template <int LAT>
__host__ __device__ constexpr bool row_used(int r) {
  for (int a = 0; a < VS<LAT>::Q; ++a)
    if (pull_row<LAT>(a) == r) return true;
  return false;
}
template <int LAT>
__host__ __device__ constexpr bool row_shifted(int r) {
  for (int a = 0; a < VS<LAT>::Q; ++a)
    if (pull_row<LAT>(a) == r && VS<LAT>::cx(a) != 0) return true;
  return false;
}

// pass 1 (float64 storage): densities -> EOS -> psi on planes [plane0, plane0 + nplanes)
// Each wavefront covers 64 cells of one row (as in the collide pass): segment
// logical_block() * (B / 64) + wavefront, B the threads per workgroup (kBlock; 64
// for small launches, see psi_small); see psi_blocks for the grid.
template <int LAT, int NC, int ST, int B = kBlock>
__global__ __launch_bounds__(B) void k_psi(KParams P, Pops<ST> in, double* __restrict__ psi, int plane0,
                                          int nplanes) {
  static_assert(ST == LBM_F64, "offset storage runs k_psi_ilv");
  using V = VS<LAT>;
  constexpr int Q = V::Q;
  const unsigned lane = threadIdx.x & 63u;
  const unsigned seg = logical_block() * (B / 64) + (unsigned)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  RowCoord c;
  bool in_row = false;
  if (!row_segment<V::D>(P, seg, plane0, nplanes, lane, &c, &in_row)) return;   // uniform per wavefront
  const unsigned cell = c.row(0, 0) + c.x(0);
  const unsigned bits = P.bb ? P.bb[cell] : 0u;   // walls: per-cell direction mask
  double rb[NC];
#pragma unroll
  for (int s = 0; s < NC; ++s) rb[s] = 0.0;
#pragma unroll 1
  for (int s = 0; s < NC; ++s) {
    const auto cv = in.comp(s, Q, P.cells);
    double v[Q];
    // every lane pulls (lanes past the row end at x = 0; all addresses in range)
    if (P.bb) {   // walls: halfway bounce-back for pulls whose source is solid; fluid cells only
      if (in_row && !(bits >> kSolidBit)) {
#pragma unroll
        for (int a = 0; a < Q; ++a)
          v[a] = pull_bb<LAT>(cv, a, bits, cell, c.row(-V::cy(a), -V::cz(a)) + c.x(-V::cx(a)), V::w(a));
      } else {
#pragma unroll
        for (int a = 0; a < Q; ++a) v[a] = 0;
      }
    } else {
#pragma unroll
      for (int a = 0; a < Q; ++a) v[a] = cv.get_row(a, c.x(-V::cx(a)), c.row(-V::cy(a), -V::cz(a)), V::w(a));
    }
    double acc = 0;
#pragma unroll
    for (int a = 0; a < Q; ++a) acc += v[a];
#pragma unroll
    for (int t = 0; t < NC; ++t)
      if (t == s) rb[t] = acc;
  }
  if (!in_row) return;
  if (bits >> kSolidBit) psi[cell] = P.psi_wall;   // solid: the wall's psi, no EOS
  else psi[cell] = eos_psi<NC>(P, rb);
}

// workgroups of k_psi for planes [plane0, plane0 + np): kBlock / 64 row segments each
inline unsigned psi_segments(const KParams& P, int np, int D) {
  return (unsigned)np * (D == 3 ? (unsigned)P.ny : 1u) * (((unsigned)P.nx + 63u) / 64u);
}
inline unsigned psi_blocks(const KParams& P, int np, int D, int B = kBlock) {
  const unsigned per = (unsigned)B / 64u;
  return xcd_grid((psi_segments(P, np, D) + per - 1) / per);
}
// small launches (fewer than 4 segments per CU of the 256) take one-wavefront
// workgroups, so that their segments spread over all CUs rather than a quarter
// of them
constexpr unsigned kSmallPsiSegments = 4u * 256u;
inline bool psi_small(const KParams& P, int np, int D) { return psi_segments(P, np, D) < kSmallPsiSegments; }

// pass 2 (float64 storage): a block is 64 cells x NC wavefronts, wavefront s
// working on component s.  Each wavefront pulls its component (rbar_s, j_s) and
// sums the psi stencil over the directions a with (a - 1) mod NC == s; the block
// combines the per-component sums through LDS in a fixed component order (rho,
// Gamma, j, F identical in every wavefront), then each wavefront splits the
// force, collides and stores component s.
constexpr int kCells = 64;

template <int LAT, int NC, int ST, int COLL, int FORC>
__global__ __launch_bounds__(kCells * 4) void k_collide(KParams P, Pops<ST> in, Pops<ST> out,
                                                       const double* __restrict__ psi, int plane0, int nplanes) {
  static_assert(ST == LBM_F64, "offset storage runs k_collide_ilv");
  using V = VS<LAT>;
  using R = double;
  constexpr int Q = V::Q;
  __shared__ double red[NC][7][kCells];
  const int lane = threadIdx.x & (kCells - 1);
  // uniform per wavefront (wave64): read it from lane 0 so it lives in a scalar register
  const int s = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kCells));
  RowCoord c;
  bool in_row = false;
  // a segment past the launch's range: the whole workgroup leaves (uniform)
  if (!row_segment<V::D>(P, logical_block(), plane0, nplanes, (unsigned)lane, &c, &in_row)) return;
  bool valid = in_row;
  const auto cv = in.comp(s, Q, P.cells);
  const rsrc_t psr = make_rsrc(psi, (unsigned)P.cells * 8u);
  const unsigned own = c.row(0, 0) + c.x(0);
  const unsigned bits = P.bb ? P.bb[own] : 0u;   // walls: per-cell direction mask
  R f[Q];
  R jx = 0, jy = 0, jz = 0;
  double mass = 0.0;
  double Fp[3] = {0.0, 0.0, 0.0};
  // every lane pulls (lanes past the row end at x = 0; all addresses in range)
  if (P.bb) {
    // walls: solid cells do not pull and do not collide; a pull whose source is
    // solid reads the cell's own opposite population (halfway bounce-back).  A
    // solid cell's slots are never read and hold zeros; its lane stores those
    // zeros again, so that every row is written whole (no partially written lines)
    valid = valid && !(bits >> kSolidBit);
    if (valid) {
#pragma unroll
      for (int a = 0; a < Q; ++a)
        f[a] = pull_bb<LAT>(cv, a, bits, own, c.row(-V::cy(a), -V::cz(a)) + c.x(-V::cx(a)), (R)V::w(a));
    } else {
#pragma unroll
      for (int a = 0; a < Q; ++a) f[a] = 0;
    }
  } else {
#pragma unroll
    for (int a = 0; a < Q; ++a) f[a] = cv.get_row(a, c.x(-V::cx(a)), c.row(-V::cy(a), -V::cz(a)), (R)V::w(a));
  }
  if (valid) {
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      mass += f[a];
      if (V::cx(a)) jx += (R)V::cx(a) * f[a];
      if (V::cy(a)) jy += (R)V::cy(a) * f[a];
      if (V::cz(a)) jz += (R)V::cz(a) * f[a];
    }
    // partial stencil of Eq. (coupledMCforce) over this wavefront's directions
    const double hb = 0.5 * (1.0 - P.beta);
    const double ps = bload(psr, c.x(0) * 8u, c.row(0, 0) * 8u, 0.0);
    static_for<1, Q>([&](auto A) {
      constexpr int a = decltype(A)::value;
      if ((a - 1) % NC == s) {
        const double pn = bload(psr, c.x(V::cx(a)) * 8u, c.row(V::cy(a), V::cz(a)) * 8u, 0.0);
        const double t = V::w(a) * pn * (P.beta * ps + hb * pn);
        if constexpr (V::cx(a) != 0) Fp[0] += V::cx(a) * t;
        if constexpr (V::cy(a) != 0) Fp[1] += V::cy(a) * t;
        if constexpr (V::cz(a) != 0) Fp[2] += V::cz(a) * t;
      }
    });
  }
  const R rs = mass;
  red[s][0][lane] = mass;
  red[s][1][lane] = jx;
  red[s][2][lane] = jy;
  red[s][3][lane] = jz;
  red[s][4][lane] = Fp[0];
  red[s][5][lane] = Fp[1];
  red[s][6][lane] = Fp[2];
  __syncthreads();
  if (!in_row) return;
  double rho = 0.0, Gam = 0.0, j[3] = {0.0, 0.0, 0.0}, F[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int t = 0; t < NC; ++t) {
    const double r = red[t][0][lane];
    rho += r;
    Gam += P.gamma[t] * r;
    j[0] += red[t][1][lane];
    j[1] += red[t][2][lane];
    j[2] += red[t][3][lane];
    F[0] += red[t][4][lane];
    F[1] += red[t][5][lane];
    F[2] += red[t][6][lane];
  }
  F[0] *= -P.G;
  F[1] *= -P.G;
  F[2] *= -P.G;
  if (valid && !(Gam > 0.0)) flag_error(P);
  R u[3], fs[3];
  cell_velocity_split<FORC>(P, s, rho, Gam, j, F, rs, u, fs);
  if (!valid) {   // a solid cell (walls): f = 0, rbar = 0 and u = du = 0 collide to zeros
    u[0] = u[1] = u[2] = 0;
    fs[0] = fs[1] = fs[2] = 0;
  }
  collide_values<LAT, R, COLL, FORC>(P, f, rs, u, fs, [&](const R* fo) {
    out.comp(s, Q, P.cells).template put_all_row<Q>(c.x(0), c.row(0, 0), fo, mass, [](int a) { return V::w(a); });
  });
}

// ---------------------------------------------------------------------------
// Component-interleaved offset storage (IlvPops): one lane = one cell with all
// its components.  Each direction's nc offsets are one vector load (float16: 2 nc
// bytes, float32: 4 nc bytes) and so are a cell's nc bases; per wavefront of 64
// cells the pull takes Q offset loads and one base load per source row, where the
// per-component layout took nc times as many.
// ---------------------------------------------------------------------------

// Dwords holding the nc values of H of one cell.
template <typename H, int NC>
struct IlvWords {
  static constexpr int N = std::is_same<H, __half>::value ? (NC + 1) / 2 : NC;
};

// Load / store the nc values of H of one cell at byte offset voff + soff.
// Float16 with nc = 3 (6 bytes) takes a dword and a 16-bit access.
template <int CP, typename H, int NC>
__device__ __forceinline__ void ilv_load(rsrc_t r, unsigned voff, unsigned soff, unsigned* w) {
  constexpr int N = IlvWords<H, NC>::N;
  if constexpr (std::is_same<H, __half>::value && NC == 3) {
    w[0] = (unsigned)__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, CP);
    w[1] = (unsigned)__builtin_amdgcn_raw_buffer_load_b16(r, voff + 4u, soff, CP);
  } else if constexpr (std::is_same<H, __half>::value && NC == 1) {
    w[0] = (unsigned)__builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, CP);
  } else if constexpr (N == 1) {
    w[0] = (unsigned)__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, CP);
  } else if constexpr (N == 2) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, CP);
    w[0] = (unsigned)v[0];
    w[1] = (unsigned)v[1];
  } else if constexpr (N == 3) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b96(r, voff, soff, CP);
    w[0] = (unsigned)v[0];
    w[1] = (unsigned)v[1];
    w[2] = (unsigned)v[2];
  } else {
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, CP);
    w[0] = (unsigned)v[0];
    w[1] = (unsigned)v[1];
    w[2] = (unsigned)v[2];
    w[3] = (unsigned)v[3];
  }
}
template <int CP, typename H, int NC>
__device__ __forceinline__ void ilv_store(rsrc_t r, unsigned voff, unsigned soff, const unsigned* w) {
  constexpr int N = IlvWords<H, NC>::N;
  if constexpr (std::is_same<H, __half>::value && NC == 3) {
    __builtin_amdgcn_raw_buffer_store_b32(w[0], r, voff, soff, CP);
    __builtin_amdgcn_raw_buffer_store_b16((unsigned short)w[1], r, voff + 4u, soff, CP);
  } else if constexpr (std::is_same<H, __half>::value && NC == 1) {
    __builtin_amdgcn_raw_buffer_store_b16((unsigned short)w[0], r, voff, soff, CP);
  } else if constexpr (N == 1) {
    __builtin_amdgcn_raw_buffer_store_b32(w[0], r, voff, soff, CP);
  } else if constexpr (N == 2) {
    decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0)) v;
    v[0] = w[0];
    v[1] = w[1];
    __builtin_amdgcn_raw_buffer_store_b64(v, r, voff, soff, CP);
  } else if constexpr (N == 3) {
    decltype(__builtin_amdgcn_raw_buffer_load_b96(r, 0, 0, 0)) v;
    v[0] = w[0];
    v[1] = w[1];
    v[2] = w[2];
    __builtin_amdgcn_raw_buffer_store_b96(v, r, voff, soff, CP);
  } else {
    decltype(__builtin_amdgcn_raw_buffer_load_b128(r, 0, 0, 0)) v;
    v[0] = w[0];
    v[1] = w[1];
    v[2] = w[2];
    v[3] = w[3];
    __builtin_amdgcn_raw_buffer_store_b128(v, r, voff, soff, CP);
  }
}
// value s of H packed in the dwords w, widened to float32
template <typename H>
__device__ __forceinline__ float ilv_get(const unsigned* w, int s) {
  if constexpr (std::is_same<H, __half>::value) {
    const unsigned short b = (unsigned short)((s & 1) ? (w[s >> 1] >> 16) : (w[s >> 1] & 0xffffu));
    return __half2float(__builtin_bit_cast(__half, b));
  } else {
    return __builtin_bit_cast(float, w[s]);
  }
}
template <typename H>
__device__ __forceinline__ void ilv_set(unsigned* w, int s, H v) {
  if constexpr (std::is_same<H, __half>::value) {
    const unsigned b = (unsigned)__builtin_bit_cast(unsigned short, v);
    if (s & 1) w[s >> 1] |= b << 16;
    else w[s >> 1] = b;
  } else {
    w[s] = __builtin_bit_cast(unsigned, v);
  }
}

// Buffer resources and strides of the interleaved planes of a box.
template <typename H, int NC, int Q>
struct IlvBufs {
  rsrc_t rb, rr;
  unsigned plane;                                   // bytes per direction plane
  static constexpr unsigned cs = NC * sizeof(H);    // bytes per cell in a plane
  static constexpr unsigned bs = NC * 4u;           // bytes per cell of the base
  __device__ __forceinline__ IlvBufs(const IlvPops<H>& p, int cells) : IlvBufs(p.base, p.r, (unsigned)cells) {}
  __device__ __forceinline__ IlvBufs(const float* base, const H* r, unsigned cells) {
    plane = cells * cs;
    rb = make_rsrc(base, cells * bs);
    rr = make_rsrc(r, (unsigned)Q * plane);
  }
};

// Pull of all components at one cell, decoded: f[s][a] = b_s(src) (w_a + r_a,s(src)).
// Row-structured (no walls): the bases of the Q sources come from one vector load
// per source row at x, with x - 1 and x + 1 taken from the neighbouring lanes (DPP
// wave shifts) and the two values past the wavefront's ends from wavefront-uniform
// scalar loads (see row_segment: lanes past a short row's end hold x = 0, the
// periodic right neighbour of its last cell).  issue() starts every load, decode()
// shifts and decodes; every lane of the wavefront must be active in decode().
// BB (walls, halfway bounce-back as in pull_bb): where the source x - e_a of a
// direction is solid (bit a of `bits`), the lane loads the offsets of its own slot
// of the opposite direction instead and decodes them with its own base (the
// unshifted value of its own row); the other bases still come from the row loads.
// Lanes with `load` false issue no offset loads (their f is undefined).
template <int LAT, int NC, typename H, bool BB = false>
struct IlvRowPull {
  static constexpr int Q = VS<LAT>::Q;
  static constexpr int NW = IlvWords<H, NC>::N;
  static constexpr int kOwnRow = 4;   // row index r = (dy + 1) + 3 (dz + 1) of (0, 0)
  unsigned bq[9][NC];
  float hl[9][NC], hr[9][NC];
  unsigned rw[Q][NW];
  __device__ __forceinline__ void issue(const IlvPops<H>& in, const IlvBufs<H, NC, Q>& B, const RowCoord& c,
                                        unsigned nx, unsigned bits = 0u, bool load = true) {
    using V = VS<LAT>;
    using IB = IlvBufs<H, NC, Q>;
    const unsigned xl = c.x0 == 0 ? nx - 1 : c.x0 - 1;
    const unsigned xr = c.x0 + 64u < nx ? c.x0 + 64u : 0u;
    static_for<0, 9>([&](auto Rr) {
      constexpr int r = decltype(Rr)::value;
      if constexpr (row_used<LAT>(r)) {
        const unsigned ro = c.row(r % 3 - 1, r / 3 - 1);
        ilv_load<0, float, NC>(B.rb, c.x(0) * IB::bs, ro * IB::bs, bq[r]);
        if constexpr (row_shifted<LAT>(r)) {
#pragma unroll
          for (int s = 0; s < NC; ++s) {
            hl[r][s] = in.base[(size_t)(ro + xl) * NC + s];
            hr[r][s] = in.base[(size_t)(ro + xr) * NC + s];
          }
        }
      }
    });
    if constexpr (BB) {
      if (load) {
        const unsigned own = (c.row(0, 0) + c.x(0)) * IB::cs;
#pragma unroll
        for (int a = 0; a < Q; ++a) {
          const unsigned off = ((bits >> a) & 1u)
                                   ? own + (unsigned)V::opp(a) * B.plane
                                   : (c.row(-V::cy(a), -V::cz(a)) + c.x(-V::cx(a))) * IB::cs + (unsigned)a * B.plane;
          ilv_load<kPopLoad, H, NC>(B.rr, off, 0u, rw[a]);
        }
      }
    } else {
#pragma unroll
      for (int a = 0; a < Q; ++a)
        ilv_load<kPopLoad, H, NC>(B.rr, c.x(-V::cx(a)) * IB::cs,
                                  (unsigned)a * B.plane + c.row(-V::cy(a), -V::cz(a)) * IB::cs, rw[a]);
    }
  }
  __device__ __forceinline__ void decode(float (&f)[NC][Q], unsigned bits = 0u) const {
    using V = VS<LAT>;
    const float one = opaque_one();
    float ob[NC];
#pragma unroll
    for (int s = 0; s < NC; ++s) ob[s] = __builtin_bit_cast(float, bq[kOwnRow][s]);
    static_for<0, Q>([&](auto A) {
      constexpr int a = decltype(A)::value;
      constexpr int r = pull_row<LAT>(a);
#pragma unroll
      for (int s = 0; s < NC; ++s) {
        const float b0 = __builtin_bit_cast(float, bq[r][s]);
        float b;
        if constexpr (V::cx(a) == 0) b = b0;
        else if constexpr (V::cx(a) > 0) b = lane_from_left(b0, hl[r][s]);   // source x - 1
        else b = lane_from_right(b0, hr[r][s]);                              // source x + 1
        if constexpr (BB && a != 0) b = ((bits >> a) & 1u) ? ob[s] : b;   // bounced: own base
        f[s][a] = b * w_plus((float)V::w(a), ilv_get<H>(rw[a], s), one);
      }
    });
  }
};

template <int LAT, int NC, typename H, bool BB = false>
__device__ __forceinline__ void ilv_pull_row(const IlvPops<H>& in, const IlvBufs<H, NC, VS<LAT>::Q>& B,
                                             const RowCoord& c, unsigned nx, float (&f)[NC][VS<LAT>::Q],
                                             unsigned bits = 0u, bool load = true) {
  IlvRowPull<LAT, NC, H, BB> p;
  p.issue(in, B, c, nx, bits, load);
  __builtin_amdgcn_sched_barrier(0);   // every load ahead of the shifts and the decode
  p.decode(f, bits);
}

// Pull of all components at one cell (one cell per lane, any lane layout): per
// direction one vector load of the source's nc offsets and one of its nc bases;
// with walls, halfway bounce-back (the source x - e_a when fluid, else the cell's
// own slot of the opposite direction).  The batched kernels and the moments use it.
template <int LAT, int NC, typename H, int CP>
__device__ __forceinline__ void ilv_pull_cell(const IlvBufs<H, NC, VS<LAT>::Q>& Bf, const Coord& c, unsigned cell,
                                              unsigned bits, bool walls, float (&f)[NC][VS<LAT>::Q]) {
  using V = VS<LAT>;
  constexpr int Q = V::Q;
  constexpr int NW = IlvWords<H, NC>::N;
  using IB = IlvBufs<H, NC, Q>;
  unsigned bw[Q][NC], rw[Q][NW];
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    const bool back = walls && ((bits >> a) & 1u);
    const unsigned src = back ? cell : c.at(-V::cx(a), -V::cy(a), -V::cz(a));
    const unsigned dir = back ? (unsigned)V::opp(a) : (unsigned)a;
    ilv_load<0, float, NC>(Bf.rb, src * IB::bs, 0u, bw[a]);
    ilv_load<CP, H, NC>(Bf.rr, src * IB::cs + dir * Bf.plane, 0u, rw[a]);
  }
  __builtin_amdgcn_sched_barrier(0);   // every load ahead of the decode
  const float one = opaque_one();
#pragma unroll
  for (int a = 0; a < Q; ++a)
#pragma unroll
    for (int s = 0; s < NC; ++s)
      f[s][a] = __builtin_bit_cast(float, bw[a][s]) * w_plus((float)V::w(a), ilv_get<H>(rw[a], s), one);
}

// pass 1 (interleaved offset storage): densities -> EOS -> psi, one cell per lane
// with all its components; row segments as in k_psi.  WALLS: the instantiation for
// boxes with solid cells (P.bb set), chosen at launch, so that the walls pull's
// registers (about 140 VGPRs, 3 wavefronts per SIMD) do not lower the occupancy of
// the plain pass (4 per SIMD).
template <int LAT, int NC, int ST, int B = kBlock, bool WALLS = false>
__global__ __launch_bounds__(B) void k_psi_ilv(KParams P, Pops<ST> in, double* __restrict__ psi, int plane0,
                                              int nplanes) {
  using V = VS<LAT>;
  using H = typename Pops<ST>::Elem;
  constexpr int Q = V::Q;
  const unsigned lane = threadIdx.x & 63u;
  const unsigned seg = logical_block() * (B / 64) + (unsigned)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  RowCoord c;
  bool in_row = false;
  if (!row_segment<V::D>(P, seg, plane0, nplanes, lane, &c, &in_row)) return;   // uniform per wavefront
  const unsigned cell = c.row(0, 0) + c.x(0);
  const unsigned bits = WALLS ? P.bb[cell] : 0u;
  const IlvBufs<H, NC, Q> Bf(in, P.cells);
  float f[NC][Q];
  if constexpr (WALLS)   // every lane takes part in the base shifts; solid lanes load no offsets
    ilv_pull_row<LAT, NC, H, true>(in, Bf, c, (unsigned)P.nx, f, bits, in_row && !(bits >> kSolidBit));
  else
    ilv_pull_row<LAT, NC, H>(in, Bf, c, (unsigned)P.nx, f);   // every lane pulls
  if (!in_row) return;
  if (bits >> kSolidBit) {   // solid: the wall's psi, no EOS
    psi[cell] = P.psi_wall;
    return;
  }
  double rb[NC];
#pragma unroll
  for (int s = 0; s < NC; ++s) {
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < Q; ++a) acc += (double)f[s][a];
    rb[s] = acc;
  }
  psi[cell] = eos_psi<NC>(P, rb);
}

// pass 2 (interleaved offset storage): one cell per lane with all its components.
// Loads psi at the cell and its Q - 1 neighbours and the pulls of every component,
// sums the stencil of Eq. (coupledMCforce), the densities and momenta, forms the
// velocity and the split, then collides and encodes each component in turn and
// stores each direction's nc offsets with one vector store.  Workgroups of
// ilv_waves(WALLS) independent row segments (wavefronts).
//
// WALLS: the instantiation for boxes with solid cells (P.bb set), chosen at launch
// (measured: both the plain and the walls collide run 2-3 % faster as separate
// instantiations).
// Wavefronts per workgroup, measured at 128^3: the plain collide 149.7 us with 4,
// 145-148 us with 2 and 1 (1 ahead by about 1 %); the walls collide 163 us with 2,
// 166 us with 1.
constexpr int ilv_waves(bool walls) { return walls ? 2 : 1; }

template <int LAT, int NC, int ST, int COLL, int FORC, bool WALLS>
__global__ __launch_bounds__(64 * ilv_waves(WALLS)) void k_collide_ilv(KParams P, Pops<ST> in, Pops<ST> out,
                                                               const double* __restrict__ psi, int plane0,
                                                               int nplanes) {
  using V = VS<LAT>;
  using H = typename Pops<ST>::Elem;
  using R = float;
  constexpr int Q = V::Q;
  constexpr int NW = IlvWords<H, NC>::N;
  using IB = IlvBufs<H, NC, Q>;
  const unsigned lane = threadIdx.x & 63u;
  const unsigned seg =
      logical_block() * ilv_waves(WALLS) + (unsigned)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  RowCoord c;
  bool in_row = false;
  if (!row_segment<V::D>(P, seg, plane0, nplanes, lane, &c, &in_row)) return;   // uniform per wavefront
  const unsigned own = c.row(0, 0) + c.x(0);
  const unsigned bits = WALLS ? P.bb[own] : 0u;
  const bool valid = in_row && !(bits >> kSolidBit);
  // psi at the cell and its neighbours first (their latency overlaps the pulls'):
  // one load per neighbour row (dy, dz), the x-neighbours by lane shifts, the
  // values past the segment's ends from scalar loads (lanes past a short row's end
  // hold x = 0, the periodic neighbour of the row's last cell)
  const rsrc_t psr = make_rsrc(psi, (unsigned)P.cells * 8u);
  double prow[9], pfl[9], pfr[9];
  {
    const unsigned nx = P.nx;
    const unsigned xl = c.x0 == 0 ? nx - 1 : c.x0 - 1;
    const unsigned xr = c.x0 + 64u < nx ? c.x0 + 64u : 0u;
    static_for<0, 9>([&](auto Rr) {
      constexpr int r = decltype(Rr)::value;
      if constexpr (row_used<LAT>(r)) {
        const unsigned ro = c.row(r % 3 - 1, r / 3 - 1);
        prow[r] = bload(psr, c.x(0) * 8u, ro * 8u, 0.0);
        if constexpr (row_shifted<LAT>(r)) {
          pfl[r] = psi[ro + xl];
          pfr[r] = psi[ro + xr];
        }
      }
    });
  }
  const IB Bi(in, P.cells);
  float f[NC][Q];
  if constexpr (WALLS) {
    // walls: solid cells load no offsets and do not collide; their slots are never
    // read and hold zeros, which their lanes store again (whole rows written)
    ilv_pull_row<LAT, NC, H, true>(in, Bi, c, (unsigned)P.nx, f, bits, valid);
    if (!valid) {
#pragma unroll
      for (int s = 0; s < NC; ++s)
#pragma unroll
        for (int a = 0; a < Q; ++a) f[s][a] = 0.0f;
    }
  } else {
    ilv_pull_row<LAT, NC, H>(in, Bi, c, (unsigned)P.nx, f);   // every lane pulls
  }
  // psi at x + e_a: row (c_y, c_z) (the pull row of the opposite velocity), shifted by c_x
  double pn[Q];
  static_for<0, Q>([&](auto A) {
    constexpr int a = decltype(A)::value;
    constexpr int r = pull_row<LAT>(V::opp(a));
    if constexpr (V::cx(a) == 0) pn[a] = prow[r];
    else if constexpr (V::cx(a) > 0) pn[a] = lane_from_right(prow[r], pfr[r]);   // x + 1
    else pn[a] = lane_from_left(prow[r], pfl[r]);                                // x - 1
  });
  if (!in_row) return;
  // total force of Eq. (coupledMCforce) (float64), summed over opposite pairs:
  // w psi_a (b psi + h psi_a) - w psi_b (b psi + h psi_b) = w (psi_a - psi_b) (b psi + h (psi_a + psi_b))
  double F[3] = {0.0, 0.0, 0.0};
  {
    const double hb = 0.5 * (1.0 - P.beta);
    const double bps = P.beta * pn[0];
    static_for<0, (Q - 1) / 2>([&](auto Pp) {
      constexpr int a = V::pair_first(decltype(Pp)::value), b = V::opp(a);
      const double t = V::w(a) * (pn[a] - pn[b]) * (bps + hb * (pn[a] + pn[b]));
      if constexpr (V::cx(a) != 0) F[0] += V::cx(a) * t;
      if constexpr (V::cy(a) != 0) F[1] += V::cy(a) * t;
      if constexpr (V::cz(a) != 0) F[2] += V::cz(a) * t;
    });
    F[0] *= -P.G;
    F[1] *= -P.G;
    F[2] *= -P.G;
  }
  // densities (float64 masses, exact for the encoding) and the momentum, summed
  // over the components of each direction first (float32, then widened)
  double mass[NC], rho = 0.0, Gam = 0.0, j[3];
#pragma unroll
  for (int s = 0; s < NC; ++s) {
    double m = 0.0;
#pragma unroll
    for (int a = 0; a < Q; ++a) m += (double)f[s][a];
    mass[s] = valid ? m : 0.0;
    rho += mass[s];
    Gam += P.gamma[s] * mass[s];
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
  if (valid && !(Gam > 0.0)) flag_error(P);
  unsigned ro[Q][NW];
  float bo[NC];
  static_for<0, NC>([&](auto S_) {
    constexpr int s = decltype(S_)::value;
    const R rs = (R)mass[s];
    R u[3], fs[3];
    cell_velocity_split<FORC>(P, s, rho, Gam, j, F, rs, u, fs);
    if (!valid) {   // a solid cell (walls): f = 0, rbar = 0 and u = du = 0 collide to zeros
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
  const IB Bo(out, P.cells);
#pragma unroll
  for (int a = 0; a < Q; ++a)
    ilv_store<kPopStore, H, NC>(Bo.rr, c.x(0) * IB::cs, (unsigned)a * Bo.plane + c.row(0, 0) * IB::cs, ro[a]);
  unsigned bw[NC];
#pragma unroll
  for (int s = 0; s < NC; ++s) bw[s] = __builtin_bit_cast(unsigned, bo[s]);
  ilv_store<kBaseStore, float, NC>(Bo.rb, c.x(0) * IB::bs, c.row(0, 0) * IB::bs, bw);
}

}  // namespace lbmk
