// Lattice velocity sets for the device kernels and the host library.
//
// D2Q9 and D3Q19 are the lattices of the paper's Section 2 (velocity sets and
// weights of Qian, d'Humieres & Lallemand 1992); D3Q7 carries the vector
// distributions of the magnetic induction solver.  Every component of a unit
// velocity is in {-1, 0, 1}; it is packed as (component + 1) in two bits per
// direction so that all lookups are integer constant expressions that fold
// away once the direction loops are unrolled.
//
// Direction order (the library's documented state-exchange order):
//   D2Q9 : 0 rest; 1 +x; 2 -x; 3 +y; 4 -y; 5 (+x,+y); 6 (-x,-y); 7 (+x,-y); 8 (-x,+y)
//   D3Q19: 0 rest; 1,2 +-x; 3,4 +-y; 5,6 +-z; 7,8 +-(x+y); 9,10 +-(x-y);
//          11,12 +-(x+z); 13,14 +-(x-z); 15,16 +-(y+z); 17,18 +-(y-z)
//   D3Q7 : 0 rest; 1,2 +-x; 3,4 +-y; 5,6 +-z
// Opposite pairs are adjacent: opp(q) = q + 1 for odd q, q - 1 for even q > 0.
#pragma once
#include <cstdint>

#ifndef __HIPCC__
#define __host__
#define __device__
#endif

namespace lbm {

constexpr uint64_t pack_dirs(const int* v, int n) {
  uint64_t r = 0;
  for (int q = 0; q < n; ++q) r |= uint64_t(v[q] + 1) << (2 * q);
  return r;
}

__host__ __device__ constexpr int unpack_dir(uint64_t code, int q) { return int((code >> (2 * q)) & 3u) - 1; }

__host__ __device__ constexpr int opp(int q) { return q == 0 ? 0 : ((q & 1) ? q + 1 : q - 1); }

namespace detail {
constexpr int d2x[9] = {0, 1, -1, 0, 0, 1, -1, 1, -1};
constexpr int d2y[9] = {0, 0, 0, 1, -1, 1, -1, -1, 1};
constexpr int d3x[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int d3y[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int d3z[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
constexpr int zeros[19] = {0};
}  // namespace detail

struct D2Q9 {
  static constexpr int Q = 9;
  static constexpr int D = 2;
  static constexpr int NC = 3;  // stress components xx, xy, yy
  static constexpr uint64_t CX = pack_dirs(detail::d2x, 9);
  static constexpr uint64_t CY = pack_dirs(detail::d2y, 9);
  static constexpr uint64_t CZ = pack_dirs(detail::zeros, 9);
  __host__ __device__ static constexpr int ex(int q) { return unpack_dir(CX, q); }
  __host__ __device__ static constexpr int ey(int q) { return unpack_dir(CY, q); }
  __host__ __device__ static constexpr int ez(int q) { return unpack_dir(CZ, q); }
  __host__ __device__ static constexpr int e2(int q) { return ex(q) * ex(q) + ey(q) * ey(q); }
  __host__ __device__ static constexpr double w(int q) { return e2(q) == 0 ? 4.0 / 9.0 : (e2(q) == 1 ? 1.0 / 9.0 : 1.0 / 36.0); }
};

struct D3Q19 {
  static constexpr int Q = 19;
  static constexpr int D = 3;
  static constexpr int NC = 6;  // xx, yy, zz, xy, xz, yz
  static constexpr uint64_t CX = pack_dirs(detail::d3x, 19);
  static constexpr uint64_t CY = pack_dirs(detail::d3y, 19);
  static constexpr uint64_t CZ = pack_dirs(detail::d3z, 19);
  __host__ __device__ static constexpr int ex(int q) { return unpack_dir(CX, q); }
  __host__ __device__ static constexpr int ey(int q) { return unpack_dir(CY, q); }
  __host__ __device__ static constexpr int ez(int q) { return unpack_dir(CZ, q); }
  __host__ __device__ static constexpr int e2(int q) { return ex(q) * ex(q) + ey(q) * ey(q) + ez(q) * ez(q); }
  __host__ __device__ static constexpr double w(int q) { return e2(q) == 0 ? 1.0 / 3.0 : (e2(q) == 1 ? 1.0 / 18.0 : 1.0 / 36.0); }
};

// Induction lattice of a flow lattice.  Its direction k is the flow
// lattice's direction k (rest, then +-x, +-y, +-z), so that wall masks and
// neighbour offsets are shared.  D3Q19 pairs with D3Q7 and three field
// components; D2Q9 with the planar restriction of D3Q7 (the two z links
// folded into the rest weight: 1/4 + 2/8 = 1/2) and the two in-plane
// components.  Both have sum_k W_k e_k e_k = theta c^2 I, theta = 1/4.
template <class L>
struct Ind;
template <>
struct Ind<D3Q19> {
  static constexpr int K = 7, NB = 3;
  __host__ __device__ static constexpr double w(int k) { return k == 0 ? 0.25 : 0.125; }
  static constexpr double theta = 0.25;
};
template <>
struct Ind<D2Q9> {
  static constexpr int K = 5, NB = 2;
  __host__ __device__ static constexpr double w(int k) { return k == 0 ? 0.5 : 0.125; }
  static constexpr double theta = 0.25;
};

}  // namespace lbm
