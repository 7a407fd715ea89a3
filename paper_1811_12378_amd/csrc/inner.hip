// Kernels of the inner preconditioner of Alg. 1 step 4 (Sec. 6.3): the regularised
// inverse of the discrete Laplacian in the sine basis, M = V diag(1 / max(lambda, 1)) V^T.
// The sine transforms V are dense contractions along each axis and run as library GEMMs
// (inner.cpp); this file holds the diagonal between them.
#include <cmath>

#include "kernels.h"

namespace hfci {
namespace {

constexpr int NT = 256;

// c[p] /= max(lambda_p, 1), lambda of the sine mode (i+1, j+1, k+1) of p = i + nx (j + ny k):
// s/h^2 * sum over axes of 2 (1 - cos(m pi / (n + 1)))
__global__ __launch_bounds__(NT) void laplace_scale_kernel(double2* __restrict__ c, int nx, int ny, int nz,
                                                           double s_h2) {
  const size_t npt = (size_t)nx * ny * nz;
  const size_t stride = (size_t)gridDim.x * NT;
  const double px = M_PI / (nx + 1), py = M_PI / (ny + 1), pz = M_PI / (nz + 1);
  for (size_t p = (size_t)blockIdx.x * NT + threadIdx.x; p < npt; p += stride) {
    const int i = (int)(p % nx), j = (int)((p / nx) % ny), k = (int)(p / ((size_t)nx * ny));
    const double lam = s_h2 * (2.0 * (1.0 - cos((i + 1) * px)) + 2.0 * (1.0 - cos((j + 1) * py)) +
                               2.0 * (1.0 - cos((k + 1) * pz)));
    const double inv = 1.0 / fmax(lam, 1.0);
    double2 v = c[p];
    v.x *= inv;
    v.y *= inv;
    c[p] = v;
  }
}

}  // namespace

void launch_laplace_scale(hipStream_t st, double2* c, const GridDesc& g) {
  const size_t npt = (size_t)g.nx * g.ny * g.nz;
  size_t b = (npt + NT - 1) / NT;
  if (b > 4096) b = 4096;
  hipLaunchKernelGGL(laplace_scale_kernel, dim3((unsigned)b), dim3(NT), 0, st, c, g.nx, g.ny, g.nz, g.s_h2);
}

}  // namespace hfci
