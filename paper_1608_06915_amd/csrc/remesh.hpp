// remesh.hpp -- state transfer between two refinement layouts of one domain (remesh.hip).
#pragma once
#include "elbm_dev.hpp"

namespace elbm {

// A value read from the old lattice: the stored state of one node, reduced to
// (rho - 1, u, fac (f - f^eq)) in a staged row.
struct TPoint {
  int32_t brick;
  uint16_t node;
  uint8_t level;
  uint8_t pad;
  double fac;
};

// A node of the new lattice and where its state comes from.
//   kind 0: the old node (a = brick, b = node) at the same level: stored values copied;
//   kind 1: the old node (a, b) one level finer: coalescence with factor fac_coal[level];
//   kind 2: reconstruction from staged rows, stencil entries [a, a + b).
struct TItem {
  int32_t brick;
  uint16_t node;
  uint8_t level;
  uint8_t kind;
  int32_t a, b;
};

struct TransferArgs {
  const TPoint *pts;
  int n_pts;
  const TItem *items;
  int n_items;
  const StencilEntry *sten;
  void *stage;  // staged rows, stage_row_width(D) values of the compute type each
  const void *src[MAXL];  // old lattice: current state buffer per level
  void *dst[MAXL];        // new lattice: current state buffer per level
  double fac_coal[MAXL];  // coalescence factor into level l (from level l + 1)
};

int launch_transfer(int D, int st, const TransferArgs &a, void *stream);

}  // namespace elbm
