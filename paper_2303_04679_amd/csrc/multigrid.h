// One-dimensional taps of the cell-based interpolation T and of its exact
// transpose (Section 2.2: interior fine cells are 3/4 of their parent plus
// 1/4 of the nearer coarse neighbour; the two end fine cells extrapolate
// linearly, 5/4 and -1/4).  Tensor products of these give T in 2-D and 3-D.
#pragma once

#include <hip/hip_runtime.h>

namespace modil {

// 1-D taps of the cell-based T: fine cell i of 2n fine cells from n coarse.
template <typename T>
__device__ inline void prolong_taps(int i, int n, int (&idx)[2], T (&w)[2]) {
  const int J = i >> 1;
  const int nb = (i & 1) ? J + 1 : J - 1;
  if (nb < 0) {
    idx[0] = J; w[0] = T(1.25); idx[1] = J + 1; w[1] = T(-0.25);
  } else if (nb >= n) {
    idx[0] = J; w[0] = T(1.25); idx[1] = J - 1; w[1] = T(-0.25);
  } else {
    idx[0] = J; w[0] = T(0.75); idx[1] = nb; w[1] = T(0.25);
  }
}

// 1-D taps of T^T: coarse cell J of n coarse cells gathers from 2n fine.
template <typename T>
__device__ inline int restrict_taps(int J, int n, int (&idx)[6], T (&w)[6]) {
  int k = 0;
  if (J >= 1) { idx[k] = 2 * J - 1; w[k++] = T(0.25); }
  idx[k] = 2 * J; w[k++] = (J == 0) ? T(1.25) : T(0.75);
  idx[k] = 2 * J + 1; w[k++] = (J == n - 1) ? T(1.25) : T(0.75);
  if (J <= n - 2) { idx[k] = 2 * J + 2; w[k++] = T(0.25); }
  if (J == 1) { idx[k] = 0; w[k++] = T(-0.25); }
  if (J == n - 2) { idx[k] = 2 * n - 1; w[k++] = T(-0.25); }
  return k;
}

// Entry of the cell-based T: weight of coarse cell J (of n) in fine cell r.
template <typename T>
__device__ inline T t_entry(int r, int J, int n) {
  if (r == 0) return J == 0 ? T(1.25) : (J == 1 ? T(-0.25) : T(0));
  if (r == 2 * n - 1) return J == n - 1 ? T(1.25) : (J == n - 2 ? T(-0.25) : T(0));
  const int K = r >> 1;
  const int nb = (r & 1) ? K + 1 : K - 1;
  return J == K ? T(0.75) : (J == nb ? T(0.25) : T(0));
}

// Column J of T as six taps: a window of four contiguous fine cells around
// 2J (clamped to the grid) and the two end fine cells, whose extrapolation
// rows reach coarse cells 1 and n-2; a slot has weight 0 when unused.
template <typename T>
__device__ inline void restrict_taps6(int J, int n, int (&idx)[6], T (&w)[6]) {
  int s = 2 * J - 1;
  s = s < 0 ? 0 : s;
  s = s > 2 * n - 4 ? 2 * n - 4 : s;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    idx[k] = s + k;
    w[k] = t_entry<T>(s + k, J, n);
  }
  idx[4] = 0;
  w[4] = s > 0 ? t_entry<T>(0, J, n) : T(0);
  idx[5] = 2 * n - 1;
  w[5] = s + 3 < 2 * n - 1 ? t_entry<T>(2 * n - 1, J, n) : T(0);
}

// Node-based T (Section 2.2): n + 1 coarse nodes -> 2n + 1 fine nodes; even
// fine nodes copy the coincident coarse node, odd ones take the mean of the
// two neighbours.  Fine node i of 2n + 1:
template <typename T>
__device__ inline void prolong_taps_node(int i, int (&idx)[2], T (&w)[2]) {
  const int J = i >> 1;
  if (i & 1) {
    idx[0] = J; w[0] = T(0.5); idx[1] = J + 1; w[1] = T(0.5);
  } else {
    idx[0] = J; w[0] = T(1); idx[1] = J; w[1] = T(0);
  }
}

// Column J of the node-based T (coarse node J of n + 1): fine nodes 2J - 1,
// 2J, 2J + 1 with weights 1/2, 1, 1/2, clamped to the grid (weight 0 outside).
template <typename T>
__device__ inline void restrict_taps_node(int J, int n_fine_nodes, int (&idx)[3], T (&w)[3]) {
  idx[1] = 2 * J; w[1] = T(1);
  idx[0] = 2 * J - 1 >= 0 ? 2 * J - 1 : 0; w[0] = 2 * J - 1 >= 0 ? T(0.5) : T(0);
  idx[2] = 2 * J + 1 < n_fine_nodes ? 2 * J + 1 : n_fine_nodes - 1;
  w[2] = 2 * J + 1 < n_fine_nodes ? T(0.5) : T(0);
}

}  // namespace modil
