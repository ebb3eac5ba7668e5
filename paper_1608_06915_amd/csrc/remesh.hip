// remesh.hip -- state transfer between two refinement layouts of one domain.
//
// Adaptive refinement, which the conclusion (Sec. V) proposes with the stabiliser's
// deviation from 2 as its criterion, changes a lattice's blocks at a coarse-step
// boundary.  The new lattice takes its state from the old one node by node: a node
// present in both keeps its stored values; a coarse node whose region is no longer
// refined is coalesced from the old finer node at its place; a node of a newly refined
// region is reconstructed by the four-point interpolation of Eq. interp from old
// values (old nodes of its own level where present, old parent nodes elsewhere).  The
// non-equilibrium part of a post-collision state scales between levels by
// beta_c (1 - 2 beta_f) / (2 beta_f (1 - 2 beta_c)) (Eq. f_neq_rescaling_iso combined
// with f' - f^eq = (1 - 2 beta)(f - f^eq) at the LBGK value gamma = 2 of resolved
// flow).  The host builds the tables (which node comes from where); the arithmetic
// runs here.
#include "lbm_device.hpp"
#include "remesh.hpp"

namespace elbm {

// one staged row per old value: (rho - 1, u, fac (h - W q)) of the stored state
template <int D, int ST> __global__ __launch_bounds__(256) void k_transfer_points(TransferArgs a) {
  using C = Codec<ST>;
  using T = typename C::T;
  constexpr int Q = nq<D>();
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.n_pts) return;
  const TPoint g = a.pts[p];
  const typename C::S *src = (const typename C::S *)a.src[g.level] + (size_t)g.brick * Q * BN + g.node;
  T h[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) h[i] = C::ld(src + (size_t)i * BN, T(wgt<D>(i)));
  T drho, j[3];
  moments<D, T>(h, drho, j);
  const T ir = T(1) / (T(1) + drho);
  const T u[3] = {j[0] * ir, j[1] * ir, j[2] * ir};
  T q[Q];
  eq_dev<D, T>(drho, u, q);
  const T fac = T(g.fac);
  T *row = (T *)a.stage + (size_t)p * stage_width<D>();
  row[0] = drho;
#pragma unroll
  for (int c = 0; c < D; ++c) row[1 + c] = u[c];
#pragma unroll
  for (int i = 0; i < Q; ++i) row[1 + D + i] = fac * (h[i] - T(wgt<D>(i)) * q[i]);
}

// one thread per node of the new lattice
template <int D, int ST> __global__ __launch_bounds__(256) void k_transfer_nodes(TransferArgs a) {
  using C = Codec<ST>;
  using S = typename C::S;
  using T = typename C::T;
  constexpr int Q = nq<D>();
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.n_items) return;
  const TItem it = a.items[t];
  S *dst = (S *)a.dst[it.level] + (size_t)it.brick * Q * BN + it.node;
  if (it.kind == 0) {  // same node: the stored values, bit for bit
    const S *src = (const S *)a.src[it.level] + (size_t)it.a * Q * BN + it.b;
#pragma unroll
    for (int i = 0; i < Q; ++i) dst[(size_t)i * BN] = src[(size_t)i * BN];
    return;
  }
  T drho, u[3] = {0, 0, 0}, n[Q];
  if (it.kind == 1) {  // coalescence of the old finer node
    const S *src = (const S *)a.src[it.level + 1] + (size_t)it.a * Q * BN + it.b;
    T h[Q], j[3];
#pragma unroll
    for (int i = 0; i < Q; ++i) h[i] = C::ld(src + (size_t)i * BN, T(wgt<D>(i)));
    moments<D, T>(h, drho, j);
    const T ir = T(1) / (T(1) + drho);
#pragma unroll
    for (int c = 0; c < 3; ++c) u[c] = j[c] * ir;
    T q[Q];
    eq_dev<D, T>(drho, u, q);
    const T fac = T(a.fac_coal[it.level]);
#pragma unroll
    for (int i = 0; i < Q; ++i) n[i] = fac * (h[i] - T(wgt<D>(i)) * q[i]);
  } else {  // reconstruction (Eq. interp) from the staged rows
    drho = T(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) n[i] = T(0);
    for (int e = it.a; e < it.a + it.b; ++e) {
      const StencilEntry se = a.sten[e];
      const T w = T(se.w);
      const T *row = (const T *)a.stage + (size_t)se.slot * stage_width<D>();
      drho += w * row[0];
#pragma unroll
      for (int c = 0; c < D; ++c) u[c] += w * row[1 + c];
#pragma unroll
      for (int i = 0; i < Q; ++i) n[i] += w * row[1 + D + i];
    }
  }
  T q[Q];
  eq_dev<D, T>(drho, u, q);
#pragma unroll
  for (int i = 0; i < Q; ++i) C::st(dst + (size_t)i * BN, T(wgt<D>(i)) * q[i] + n[i], T(wgt<D>(i)));
}

int launch_transfer(int D, int st, const TransferArgs &a, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  const int gp = (a.n_pts + 255) / 256, gi = (a.n_items + 255) / 256;
#define TRANSFER_LAUNCH(DD, SS)                                                            \
  do {                                                                                     \
    if (gp > 0) k_transfer_points<DD, SS><<<gp, 256, 0, s>>>(a);                           \
    if (gi > 0) k_transfer_nodes<DD, SS><<<gi, 256, 0, s>>>(a);                            \
  } while (0)
  if (D == 2) {
    switch (st) {
      case ST_F64: TRANSFER_LAUNCH(2, ST_F64); break;
      case ST_F32: TRANSFER_LAUNCH(2, ST_F32); break;
      case ST_F16S: TRANSFER_LAUNCH(2, ST_F16S); break;
      default: TRANSFER_LAUNCH(2, ST_BF16S); break;
    }
  } else {
    switch (st) {
      case ST_F64: TRANSFER_LAUNCH(3, ST_F64); break;
      case ST_F32: TRANSFER_LAUNCH(3, ST_F32); break;
      case ST_F16S: TRANSFER_LAUNCH(3, ST_F16S); break;
      default: TRANSFER_LAUNCH(3, ST_BF16S); break;
    }
  }
#undef TRANSFER_LAUNCH
  return (int)hipGetLastError();
}

}  // namespace elbm
