// Velocity sets, weights and compile-time helpers for the gfx950 kernels.
//
// The velocity order is the order of the D3Q19/D3Q27 tables of Section 2 of
// Geller, Uphoff & Krafczyk (arXiv:1206.0389); it is also the population
// order at the C ABI. D3Q27 indices 0..18 are the D3Q19 set.
#pragma once

#include <cstdint>

namespace lbm {

struct VelocitySet27 {
  static constexpr int ex[27] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1,
                                 -1, 0, 0, 0, 0, 1, -1, 1, 1, -1, -1, 1, -1};
  static constexpr int ey[27] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0,
                                 0, 1, -1, 1, -1, 1, 1, -1, 1, -1, 1, -1, -1};
  static constexpr int ez[27] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1,
                                 1, 1, -1, -1, 1, 1, 1, 1, -1, 1, -1, -1, -1};
};

constexpr int cx(int i) { return VelocitySet27::ex[i]; }
constexpr int cy(int i) { return VelocitySet27::ey[i]; }
constexpr int cz(int i) { return VelocitySet27::ez[i]; }
constexpr int c_axis(int i, int d) { return d == 0 ? cx(i) : (d == 1 ? cy(i) : cz(i)); }

constexpr int nonzero_components(int i) {
  return (cx(i) != 0) + (cy(i) != 0) + (cz(i) != 0);
}

// Quadrature weights (Section 2): by the number of non-zero components.
template <int Q>
constexpr double weight(int i) {
  return Q == 19 ? (nonzero_components(i) == 0   ? 1.0 / 3.0
                    : nonzero_components(i) == 1 ? 1.0 / 18.0
                                                 : 1.0 / 36.0)
                 : (nonzero_components(i) == 0   ? 8.0 / 27.0
                    : nonzero_components(i) == 1 ? 2.0 / 27.0
                    : nonzero_components(i) == 2 ? 1.0 / 54.0
                                                 : 1.0 / 216.0);
}

template <int Q>
constexpr int opposite(int i) {
  for (int j = 0; j < Q; ++j)
    if (cx(j) == -cx(i) && cy(j) == -cy(i) && cz(j) == -cz(i)) return j;
  return -1;
}

// Largest index distance between a population and its opposite in the
// paper's order (D3Q27: 7, for the corner pairs 19-26; D3Q19: 1). Kernels
// that address a population and its opposite from the lower of the two
// slabs span this many slabs plus one.
template <int Q>
constexpr int max_opposite_distance() {
  int d = 0;
  for (int i = 0; i < Q; ++i) {
    const int k = i - opposite<Q>(i);
    d = k > d ? k : (-k > d ? -k : d);
  }
  return d;
}

// Index of velocity (ex, ey, ez) in the D3Q27 order (-1 if absent).
constexpr int index_of(int x, int y, int z) {
  for (int j = 0; j < 27; ++j)
    if (cx(j) == x && cy(j) == y && cz(j) == z) return j;
  return -1;
}

// Direction i with the components of the axes in mask m (bit d: axis d)
// reversed: the specular image of i across faces normal to those axes.
constexpr int mirror_index(int i, int m) {
  return index_of((m & 1) ? -cx(i) : cx(i), (m & 2) ? -cy(i) : cy(i), (m & 4) ? -cz(i) : cz(i));
}

// Face bits: bit 2d is the "-" face of axis d (coordinate 0), bit 2d+1 the
// "+" face (coordinate n-1). pull_faces(i): faces crossed by x - e_i when x
// lies on them, i.e. the faces through which population i enters.
constexpr uint32_t pull_faces(int i) {
  uint32_t m = 0;
  for (int d = 0; d < 3; ++d) {
    if (c_axis(i, d) == 1) m |= 1u << (2 * d);
    if (c_axis(i, d) == -1) m |= 1u << (2 * d + 1);
  }
  return m;
}
// Faces crossed by x + e_i: the faces through which population i leaves.
constexpr uint32_t push_faces(int i) {
  uint32_t m = 0;
  for (int d = 0; d < 3; ++d) {
    if (c_axis(i, d) == 1) m |= 1u << (2 * d + 1);
    if (c_axis(i, d) == -1) m |= 1u << (2 * d);
  }
  return m;
}

}  // namespace lbm
