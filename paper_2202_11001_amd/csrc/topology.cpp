// Mesh topology of the dual simplex-mesh model (Sec. 2.1, Fig. 1 A/B):
// every cube of 8 neighbouring grid points is split into 6 tetrahedra, and the
// cubes of each 2x2x2 group are mirrored so that the split has no preferred
// direction.  The 6 tetrahedra of a cube are its monotone paths from one corner
// to the opposite one (one per ordering of the three axes); the mirrored cube
// starts its paths at the mirrored corner.
#include <stdint.h>

#include <algorithm>
#include <unordered_map>

#include "dsm_internal.h"

namespace dsm {

namespace {
// axis orderings of the monotone paths, lexicographic: xyz xzy yxz yzx zxy zyx
constexpr int kOrder[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
// parity of each ordering (number of transpositions from xyz)
constexpr int kOddOrder[6] = {0, 1, 1, 0, 0, 1};
}  // namespace

bool build_topology(const int mesh[3], HostTopology& tp) {
  const int nx = mesh[0], ny = mesh[1], nz = mesh[2];
  if (nx < 2 || ny < 2 || nz < 2) return false;
  tp.P = nx * ny * nz;
  tp.C = (nx - 1) * (ny - 1) * (nz - 1);
  tp.T = 6 * tp.C;
  tp.tets.assign(4 * (size_t)tp.T, 0);
  for (int ck = 0; ck + 1 < nz; ++ck)
    for (int cj = 0; cj + 1 < ny; ++cj)
      for (int ci = 0; ci + 1 < nx; ++ci) {
        const int cell[3] = {ci, cj, ck};
        const int flip[3] = {ci & 1, cj & 1, ck & 1};
        const int cube = ci + (nx - 1) * (cj + (ny - 1) * ck);
        for (int o = 0; o < 6; ++o) {
          int local[3] = {0, 0, 0};
          int v[4];
          for (int step = 0; step < 4; ++step) {
            if (step) local[kOrder[o][step - 1]] = 1;
            int g[3];
            for (int a = 0; a < 3; ++a) g[a] = cell[a] + (flip[a] ? 1 - local[a] : local[a]);
            v[step] = g[0] + nx * (g[1] + ny * g[2]);
          }
          // The path along xyz in an unmirrored cube is right-handed; every
          // transposition of the axis order and every mirrored axis flips the
          // handedness.  Left-handed tetrahedra get their last two vertices swapped.
          if ((kOddOrder[o] + flip[0] + flip[1] + flip[2]) & 1) std::swap(v[2], v[3]);
          int* dst = &tp.tets[4 * (size_t)(6 * cube + o)];
          for (int q = 0; q < 4; ++q) dst[q] = v[q];
        }
      }
  // edge multiplicities k_e (tetrahedra sharing each edge), for the 1/k_e
  // weights that make the per-tetrahedron deformation terms sum to one count
  // per edge (Sec. 2.3.2)
  static const int kPair[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
  std::unordered_map<uint64_t, int> mult;
  mult.reserve(8 * (size_t)tp.T);
  auto key = [](int a, int b) {
    if (a > b) std::swap(a, b);
    return ((uint64_t)(uint32_t)a << 32) | (uint32_t)b;
  };
  for (int t = 0; t < tp.T; ++t)
    for (auto& pr : kPair) mult[key(tp.tets[4 * t + pr[0]], tp.tets[4 * t + pr[1]])]++;
  tp.E = (int)mult.size();
  tp.tet_w.assign(6 * (size_t)tp.T, 0.0);
  for (int t = 0; t < tp.T; ++t)
    for (int e = 0; e < 6; ++e)
      tp.tet_w[6 * t + e] = 1.0 / mult[key(tp.tets[4 * t + kPair[e][0]], tp.tets[4 * t + kPair[e][1]])];
  // stars: tetrahedra incident to each point (Sec. 2.2), ascending
  tp.star_off.assign(tp.P + 1, 0);
  for (int i = 0; i < 4 * tp.T; ++i) tp.star_off[tp.tets[i] + 1]++;
  for (int p = 0; p < tp.P; ++p) tp.star_off[p + 1] += tp.star_off[p];
  tp.star.assign(4 * (size_t)tp.T, 0);
  std::vector<int> pos(tp.star_off.begin(), tp.star_off.end() - 1);
  for (int t = 0; t < tp.T; ++t)
    for (int q = 0; q < 4; ++q) tp.star[pos[tp.tets[4 * t + q]]++] = t;
  tp.max_star = 0;
  for (int p = 0; p < tp.P; ++p) tp.max_star = std::max(tp.max_star, tp.star_off[p + 1] - tp.star_off[p]);
  return true;
}

// Undeformed grid: n points spread over the image box [-0.5, D-0.5]; point i
// sits at lattice position i*128*D/(n-1), rounded half up.
void identity_grid(const int mesh[3], const int dims[3], float* X) {
  for (int k = 0; k < mesh[2]; ++k)
    for (int j = 0; j < mesh[1]; ++j)
      for (int i = 0; i < mesh[0]; ++i) {
        const int idx[3] = {i, j, k};
        float* dst = X + 3 * (size_t)(i + mesh[0] * (j + mesh[1] * k));
        for (int a = 0; a < 3; ++a) {
          const int64_t den = 2 * (int64_t)(mesh[a] - 1);
          const int64_t u = (256 * (int64_t)idx[a] * dims[a] + mesh[a] - 1) / den;
          dst[a] = (float)((double)u / kLat - 0.5);
        }
      }
}

}  // namespace dsm
