// Host construction of the per-cell wall masks read by the step kernels: bit a of
// cell x is set when the source x - e_a of direction a is solid (the pull then
// bounces back), bit 31 when x itself is solid.  Periodic box, x fastest.
#pragma once
#include "lattice.hpp"

namespace lbmk {

template <int LAT>
void wall_bits(long nx, long ny, long nz, const unsigned char* solid, unsigned* bits) {
  using V = VS<LAT>;
  for (long z = 0; z < nz; ++z)
    for (long y = 0; y < ny; ++y)
      for (long x = 0; x < nx; ++x) {
        const long cell = (z * ny + y) * nx + x;
        unsigned b = solid[cell] ? (1u << 31) : 0u;
        for (int a = 1; a < V::Q; ++a) {
          const long sx = (x - V::cx(a) + nx) % nx, sy = (y - V::cy(a) + ny) % ny, sz = (z - V::cz(a) + nz) % nz;
          if (solid[(sz * ny + sy) * nx + sx]) b |= 1u << a;
        }
        bits[cell] = b;
      }
}

}  // namespace lbmk
