// Point interpolants of the string's transverse nodes, shared by the host
// planner and the batched kernels of libstringfdtd (private to the library).
#pragma once
#include <hip/hip_runtime.h>

namespace sfd {

// Cubic Lagrange interpolant at x (Sec. 3.3's p-th order interpolant with
// p = 3) on the nodes l-1 .. l+2 around x = (l + a) h, as up to four distinct
// interior nodes (1-based, 0 = absent) and weights: the end nodes are fixed,
// a node past an end stands for its mirror image with sign s (-1 simply
// supported, +1 clamped: the ghosts of the boundary conditions).
__host__ __device__ inline void cubic_interp(double x, int N, double s, int n[4], double w[4]) {
  const int l = (int)floor(x * N);
  const double a = x * N - l;
  const double lw[4] = {-a * (a - 1.0) * (a - 2.0) / 6.0, (a + 1.0) * (a - 1.0) * (a - 2.0) / 2.0,
                        -(a + 1.0) * a * (a - 2.0) / 2.0, (a + 1.0) * a * (a - 1.0) / 6.0};
  for (int k = 0; k < 4; ++k) {
    n[k] = 0;
    w[k] = 0.0;
  }
  int used = 0;
  for (int k = 0; k < 4; ++k) {
    int m = l - 1 + k;
    double c = lw[k];
    if (m == -1) {
      m = 1;
      c *= s;
    } else if (m == N + 1) {
      m = N - 1;
      c *= s;
    }
    if (m < 1 || m > N - 1) continue;
    int j = 0;
    while (j < used && n[j] != m) ++j;
    if (j == used) n[used++] = m;
    w[j] += c;
  }
}

}  // namespace sfd
