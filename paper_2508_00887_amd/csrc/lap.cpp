// Exact linear assignment for the discretisation of Algorithm 1, step 10:
// M = argmin_{P in Pi} ||P - N||_F = argmax_P <P, N> (eq. 2), which the paper
// solves with the Hungarian method (Sec. 6, complexity paragraph).
//
// This is the shortest-augmenting-path form of the Hungarian method with row
// and column potentials (dual variables u, v; reduced cost c_ij - u_i - v_j
// >= 0, tight on assigned pairs).  It starts from the dual-feasible partial
// matching given by the row maxima, which the device already computed, so
// only rows whose maximum collides with another row need an augmenting path;
// each augmentation is a dense O(n^2) Dijkstra over the columns.
#include <cmath>
#include <limits>
#include <vector>

#include "fram_internal.h"

namespace fram {

void host_lap_max(const float* W, int n, int ld, const int32_t* sigma_init, int32_t* sigma) {
  const double inf = std::numeric_limits<double>::infinity();
  auto cost = [&](int i, int j) { return -(double)W[(size_t)i * ld + j]; };

  std::vector<double> u(n), v(n, 0.0), dist(n);
  std::vector<int> row_of(n, -1), col_of(n, -1), pred(n), scanned_list;
  std::vector<char> scanned(n);
  scanned_list.reserve(n);

  // Dual start: u_i = min_j c_ij, v = 0, so every row's best column is tight.
  for (int i = 0; i < n; ++i) {
    double m = inf;
    for (int j = 0; j < n; ++j) m = std::min(m, cost(i, j));
    u[i] = m;
  }
  // Keep the given (tight) assignments that do not collide.
  if (sigma_init != nullptr) {
    for (int i = 0; i < n; ++i) {
      const int j = sigma_init[i];
      if (j < 0 || j >= n || row_of[j] != -1) continue;
      if (cost(i, j) - u[i] - v[j] != 0.0) continue;
      row_of[j] = i;
      col_of[i] = j;
    }
  }

  for (int i0 = 0; i0 < n; ++i0) {
    if (col_of[i0] != -1) continue;
    for (int j = 0; j < n; ++j) {
      dist[j] = cost(i0, j) - u[i0] - v[j];
      pred[j] = i0;
      scanned[j] = 0;
    }
    scanned_list.clear();
    int jend = -1;
    double D = 0.0;
    while (true) {
      int jmin = -1;
      double dmin = inf;
      for (int j = 0; j < n; ++j)
        if (!scanned[j] && dist[j] < dmin) {
          dmin = dist[j];
          jmin = j;
        }
      if (jmin < 0) break;  // cannot happen for a complete bipartite graph
      scanned[jmin] = 1;
      scanned_list.push_back(jmin);
      if (row_of[jmin] == -1) {
        jend = jmin;
        D = dmin;
        break;
      }
      const int i = row_of[jmin];
      for (int j = 0; j < n; ++j) {
        if (scanned[j]) continue;
        const double nd = dmin + cost(i, j) - u[i] - v[j];
        if (nd < dist[j]) {
          dist[j] = nd;
          pred[j] = i;
        }
      }
    }
    if (jend < 0) break;
    // Potential update keeps reduced costs >= 0 and makes the path tight.
    u[i0] += D;
    for (int j : scanned_list) {
      if (j == jend) continue;
      const int i = row_of[j];
      v[j] += dist[j] - D;
      u[i] += D - dist[j];
    }
    // Augment along the predecessor chain.
    int j = jend;
    while (true) {
      const int i = pred[j];
      const int jprev = col_of[i];
      row_of[j] = i;
      col_of[i] = j;
      if (i == i0) break;
      j = jprev;
    }
  }
  for (int i = 0; i < n; ++i) sigma[i] = col_of[i];
}

}  // namespace fram
