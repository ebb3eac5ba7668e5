// indicator.hip -- under-resolution indicator from the entropic stabiliser.
//
// With enough resolution the stabiliser gamma of Eq. gamma_min_approx tends to its LBGK
// value 2, so its deviation measures under-resolution (Sec. IV, turbulent channel flow,
// the gamma snapshot); the conclusion (Sec. V) names that deviation as the natural
// criterion for adaptive refinement.  This file reduces it per brick: the largest
// |gamma - 2| over a brick's fluid nodes, from the per-node gamma of the last collision.
#include "indicator.hpp"
#include "lbm_device.hpp"

namespace elbm {

// One workgroup per brick of the level: each lane takes its node's |gamma - 2| (or -1
// for a node that is absent, solid or outside the level box), the workgroup keeps the
// largest, and lane 0 stores it at the brick's place in the dense brick grid.
template <int D> __global__ __launch_bounds__(BN) void k_gamma_indicator(const LevelStatic *lev, int level,
                                                                         const int32_t *borg, Dims box, Dims grid,
                                                                         float *out) {
  __shared__ float part[BN / 64];
  const int b = blockIdx.x, n = threadIdx.x;
  const LevelStatic &L = lev[level];
  int x, y, z;
  node_xyz<D>(n, x, y, z);
  const int64_t X = borg[3 * b] + x, Y = borg[3 * b + 1] + y, Z = borg[3 * b + 2] + z;
  float v = -1.0f;
  if (L.gamma && (L.cls[(size_t)b * BN + n] & CLS_FLUID) && X < box.n[0] && Y < box.n[1] && Z < box.n[2])
    v = fabsf(L.gamma[(size_t)b * BN + n] - 2.0f);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  if ((n & 63) == 0) part[n >> 6] = v;
  __syncthreads();
  if (n == 0) {
    float m = part[0];
#pragma unroll
    for (int w = 1; w < BN / 64; ++w) m = fmaxf(m, part[w]);
    const int64_t gx = borg[3 * b] / Brick<D>::BX, gy = borg[3 * b + 1] / Brick<D>::BY,
                  gz = D == 3 ? borg[3 * b + 2] / Brick<3>::BZ : 0;
    out[gx + grid.n[0] * (gy + grid.n[1] * gz)] = m;
  }
}

__global__ void k_fill_float(float *p, int64_t count, float v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (; i < count; i += step) p[i] = v;
}

int launch_gamma_indicator(int D, const LevelStatic *lev_dev, int level, int nbricks, const int32_t *borg, Dims box,
                           Dims grid, float *out, void *stream) {
  const int64_t cells = grid.n[0] * grid.n[1] * grid.n[2];
  if (cells > 0) {
    const int64_t blocks = std::min<int64_t>((cells + 255) / 256, 65536);
    k_fill_float<<<(int)blocks, 256, 0, (hipStream_t)stream>>>(out, cells, -1.0f);
  }
  if (nbricks > 0) {
    if (D == 2)
      k_gamma_indicator<2><<<nbricks, BN, 0, (hipStream_t)stream>>>(lev_dev, level, borg, box, grid, out);
    else
      k_gamma_indicator<3><<<nbricks, BN, 0, (hipStream_t)stream>>>(lev_dev, level, borg, box, grid, out);
  }
  return (int)hipGetLastError();
}

}  // namespace elbm
