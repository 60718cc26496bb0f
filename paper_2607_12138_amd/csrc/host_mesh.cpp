// Structured simplicial meshes, SplitMix64 jitter and the canonical
// local-to-global map (host side).  Compiled with -ffp-contract=off so the
// coordinates are reproducible bit for bit from their definition.
#include <algorithm>
#include <array>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <vector>

#include "internal.h"

namespace bras {

static uint64_t mix64(uint64_t z) {
  // SplitMix64 output function (Steele, Lea, Flood 2014; Vigna's constants)
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static const uint64_t kGamma = 0x9E3779B97F4A7C15ULL;

int nsym_of(int dim) { return dim * (dim + 1) / 2; }

static int64_t binom(int64_t n, int64_t k) {
  if (k < 0 || n < k) return 0;
  int64_t r = 1;
  for (int64_t i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

// DOFs per vertex, edge, face, cell of the supported families.
int element_counts(int family, int dim, int degree, int* n_loc, int counts[4]) {
  for (int i = 0; i < 4; ++i) counts[i] = 0;
  if (dim != 2 && dim != 3) return fail(BRAS_EINVAL, "dim must be 2 or 3 (got %d)", dim);
  int p = degree;
  if (family == BRAS_H1 || family == BRAS_H1_BERNSTEIN) {
    if (p < 1 || p > 6) return fail(BRAS_EINVAL, "H1 degree must be 1..6 (got %d)", p);
    counts[0] = 1;
    counts[1] = p - 1;
    if (dim == 2) {
      counts[2] = (int)binom(p - 1, 2);
    } else {
      counts[2] = (int)binom(p - 1, 2);
      counts[3] = (int)binom(p - 1, 3);
    }
    *n_loc = (int)binom(p + dim, dim);
  } else if (family == BRAS_HDIV) {
    if (p < 1 || p > 4) return fail(BRAS_EINVAL, "HDIV degree must be 1..4 (got %d)", p);
    if (dim == 2) {
      counts[1] = p;                                   // normal moments against P_{k-1}
      counts[2] = 2 * (int)binom(p - 2 + 2, 2);        // [P_{k-2}]^2
      *n_loc = 3 * counts[1] + counts[2];
    } else {
      counts[2] = (int)binom(p - 1 + 2, 2);            // P_{k-1} on the face
      counts[3] = 3 * (int)binom(p - 2 + 3, 3);        // [P_{k-2}]^3
      *n_loc = 4 * counts[2] + counts[3];
    }
  } else if (family == BRAS_HCURL) {
    if (p < 1 || p > 4) return fail(BRAS_EINVAL, "HCURL degree must be 1..4 (got %d)", p);
    counts[1] = p;                                     // tangential moments against P_{k-1}
    if (dim == 2) {
      counts[2] = 2 * (int)binom(p - 2 + 2, 2);
      *n_loc = 3 * counts[1] + counts[2];
    } else {
      counts[2] = 2 * (int)binom(p - 2 + 2, 2);        // two tangents x P_{k-2}
      counts[3] = 3 * (int)binom(p - 3 + 3, 3);        // [P_{k-3}]^3
      *n_loc = 6 * counts[1] + 4 * counts[2] + counts[3];
    }
  } else if (family == BRAS_HCURL2 || family == BRAS_HDIV2) {
    if (p < 1 || p > (dim == 2 ? 7 : 4))
      return fail(BRAS_EINVAL, "second-kind degree must be 1..%d in %dD (got %d)", dim == 2 ? 7 : 4, dim, p);
    const int rt2 = (p - 1) * (p + 1);                 // dim RT_{k-1} (2D)
    if (dim == 2) {
      counts[1] = p + 1;                               // tangential / normal moments against P_k
      counts[2] = rt2;                                 // RT_{k-1} (N2curl) or N1curl_{k-1} (BDM), same dim
      *n_loc = 3 * counts[1] + counts[2];
    } else if (family == BRAS_HCURL2) {
      counts[1] = p + 1;                               // tangential moments against P_k
      counts[2] = rt2;                                 // against RT_{k-1} on the face
      counts[3] = (p - 2) * (p - 1) * (p + 1) / 2;     // against RT_{k-2}
      *n_loc = 6 * counts[1] + 4 * counts[2] + counts[3];
    } else {
      counts[2] = (p + 1) * (p + 2) / 2;               // normal moments against P_k on the face
      counts[3] = (p - 1) * (p + 1) * (p + 2) / 2;     // against N1curl_{k-1}
      *n_loc = 4 * counts[2] + counts[3];
    }
  } else {
    return fail(BRAS_EINVAL, "unknown family %d", family);
  }
  return BRAS_OK;
}

}  // namespace bras

using namespace bras;

extern "C" int bras_mesh_size(int dim, int N, int64_t* nvert_h, int64_t* ncell_h) {
  clear_error();
  BRAS_CHECK(dim == 2 || dim == 3, "dim must be 2 or 3 (got %d)", dim);
  BRAS_CHECK(N >= 1 && N <= 2000, "N must be in [1, 2000] (got %d)", N);
  BRAS_CHECK(nvert_h && ncell_h, "null output pointer");
  int64_t n1 = N + 1;
  *nvert_h = dim == 2 ? n1 * n1 : n1 * n1 * n1;
  *ncell_h = dim == 2 ? 2LL * N * N : 6LL * N * N * N;
  return BRAS_OK;
}

extern "C" int bras_mesh_structured(int dim, int N, double jitter, uint64_t seed,
                                    double* coords_h, int32_t* cells_h) {
  int64_t nv, nc;
  int st = bras_mesh_size(dim, N, &nv, &nc);
  if (st) return st;
  BRAS_CHECK(coords_h && cells_h, "null output pointer");
  BRAS_CHECK(jitter >= 0.0 && jitter < 0.25, "jitter must be in [0, 0.25) (got %g)", jitter);
  BRAS_CHECK(nv < (1LL << 31), "mesh too large for int32 vertex ids");
  const int64_t n1 = N + 1;
  const double h = 1.0 / (double)N;
  const double amp = jitter * h;
  for (int64_t v = 0; v < nv; ++v) {
    int64_t lat[3] = {v % n1, (v / n1) % n1, (v / (n1 * n1)) % n1};
    bool interior = true;
    for (int a = 0; a < dim; ++a) interior = interior && lat[a] > 0 && lat[a] < N;
    for (int a = 0; a < dim; ++a) {
      double x = (double)lat[a] * h;
      if (jitter != 0.0 && interior) {
        uint64_t counter = (uint64_t)dim * (uint64_t)v + (uint64_t)a + 1ULL;
        uint64_t z = mix64(seed + counter * kGamma);
        double u = (double)(z >> 11) * 0x1.0p-53;
        double t = 2.0 * u;
        t = t - 1.0;
        double jit = amp * t;
        double base = (double)lat[a] * h;
        x = base + jit;
      }
      coords_h[v * dim + a] = x;
    }
  }
  if (dim == 2) {
    for (int64_t j = 0; j < N; ++j)
      for (int64_t i = 0; i < N; ++i) {
        int64_t c = i + N * j;
        int32_t v00 = (int32_t)(i + n1 * j), v10 = v00 + 1, v01 = v00 + (int32_t)n1, v11 = v01 + 1;
        int32_t* t0 = cells_h + 6 * c;
        t0[0] = v00; t0[1] = v10; t0[2] = v11;
        t0[3] = v00; t0[4] = v01; t0[5] = v11;
      }
  } else {
    static const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    const int64_t stride[3] = {1, n1, n1 * n1};
    for (int64_t k = 0; k < N; ++k)
      for (int64_t j = 0; j < N; ++j)
        for (int64_t i = 0; i < N; ++i) {
          int64_t c = i + N * (j + N * k);
          int64_t base = i + n1 * (j + n1 * k);
          for (int s = 0; s < 6; ++s) {
            int32_t* t = cells_h + 4 * (6 * c + s);
            int64_t cur = base;
            t[0] = (int32_t)cur;
            for (int q = 0; q < 3; ++q) {
              cur += stride[perms[s][q]];
              t[q + 1] = (int32_t)cur;
            }
          }
        }
  }
  return BRAS_OK;
}

extern "C" int bras_element_info(int family, int dim, int degree, int* n_loc_h, int* dofs_per_entity_h) {
  clear_error();
  BRAS_CHECK(n_loc_h && dofs_per_entity_h, "null output pointer");
  int counts[4];
  int st = element_counts(family, dim, degree, n_loc_h, counts);
  if (st) return st;
  for (int i = 0; i < 4; ++i) dofs_per_entity_h[i] = counts[i];
  return BRAS_OK;
}

namespace {

// Unique sorted entities of dimension k (k+1 vertices) and, per cell, the
// index of each local entity (local entities in lex order of local vertices).
template <int K>
void number_entities(int64_t ncell, int nv, const int32_t* cells, std::vector<std::array<int32_t, K>>& uniq,
                     std::vector<int64_t>& local_idx, int& nlocal) {
  std::vector<std::array<int, K>> combos;
  std::array<int, K> cur;
  // enumerate combinations of K out of nv in lexicographic order
  for (int i = 0; i < K; ++i) cur[i] = i;
  while (true) {
    combos.push_back(cur);
    int pos = K - 1;
    while (pos >= 0 && cur[pos] == nv - K + pos) --pos;
    if (pos < 0) break;
    ++cur[pos];
    for (int q = pos + 1; q < K; ++q) cur[q] = cur[q - 1] + 1;
  }
  nlocal = (int)combos.size();
  std::vector<std::array<int32_t, K>> keys((size_t)ncell * nlocal);
  for (int64_t c = 0; c < ncell; ++c)
    for (int e = 0; e < nlocal; ++e)
      for (int q = 0; q < K; ++q) keys[(size_t)c * nlocal + e][q] = cells[c * nv + combos[e][q]];
  uniq = keys;
  std::sort(uniq.begin(), uniq.end());
  uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
  local_idx.resize(keys.size());
  for (size_t t = 0; t < keys.size(); ++t)
    local_idx[t] = std::lower_bound(uniq.begin(), uniq.end(), keys[t]) - uniq.begin();
}

}  // namespace

extern "C" int bras_dofmap(int family, int dim, int degree, int64_t nvert, int64_t ncell,
                           const int32_t* cells_h, int64_t* n_h, int32_t* l2g_h) {
  clear_error();
  BRAS_CHECK(cells_h && n_h && l2g_h, "null pointer argument");
  BRAS_CHECK(nvert > 0 && ncell > 0, "empty mesh");
  int nl, counts[4];
  int st = element_counts(family, dim, degree, &nl, counts);
  if (st) return st;
  const int nv = dim + 1;
  for (int64_t c = 0; c < ncell; ++c)
    for (int q = 0; q < nv; ++q) {
      int32_t v = cells_h[c * nv + q];
      BRAS_CHECK(v >= 0 && v < nvert, "cell %lld vertex %d out of range", (long long)c, v);
      if (q) BRAS_CHECK(cells_h[c * nv + q - 1] < v, "cell %lld vertices not ascending", (long long)c);
    }
  // per entity dimension: number of entities and per-cell local indices
  std::vector<int64_t> ent_count(dim + 1);
  std::vector<std::vector<int64_t>> loc(dim + 1);
  std::vector<int> nlocal(dim + 1);
  ent_count[0] = nvert;
  nlocal[0] = nv;
  loc[0].resize((size_t)ncell * nv);
  for (int64_t c = 0; c < ncell; ++c)
    for (int q = 0; q < nv; ++q) loc[0][(size_t)c * nv + q] = cells_h[c * nv + q];
  ent_count[dim] = ncell;
  nlocal[dim] = 1;
  loc[dim].resize(ncell);
  std::iota(loc[dim].begin(), loc[dim].end(), 0);
  if (counts[1]) {
    std::vector<std::array<int32_t, 2>> u;
    number_entities<2>(ncell, nv, cells_h, u, loc[1], nlocal[1]);
    ent_count[1] = (int64_t)u.size();
  }
  if (dim == 3 && counts[2]) {
    std::vector<std::array<int32_t, 3>> u;
    number_entities<3>(ncell, nv, cells_h, u, loc[2], nlocal[2]);
    ent_count[2] = (int64_t)u.size();
  }
  std::vector<int64_t> offset(dim + 2, 0);
  for (int e = 0; e <= dim; ++e) offset[e + 1] = offset[e] + ent_count[e] * counts[e];
  const int64_t n = offset[dim + 1];
  BRAS_CHECK(n < (1LL << 31), "too many DOFs for int32 maps (%lld)", (long long)n);
  for (int64_t c = 0; c < ncell; ++c) {
    int col = 0;
    for (int e = 0; e <= dim; ++e) {
      int k = counts[e];
      if (!k) continue;
      for (int le = 0; le < nlocal[e]; ++le) {
        int64_t ent = loc[e][(size_t)c * nlocal[e] + le];
        for (int j = 0; j < k; ++j) l2g_h[c * nl + col++] = (int32_t)(offset[e] + ent * k + j);
      }
    }
    if (col != nl) return fail(BRAS_EINVAL, "internal: local DOF count mismatch (%d vs %d)", col, nl);
  }
  *n_h = n;
  return BRAS_OK;
}
