// elbm.cpp -- host runtime and C ABI of the refined KBC lattice Boltzmann library.
//
// Geometry (Sec. III): a level's region is the union of its blocks; child nodes at
// fine Chebyshev distance 0 / 1 from the region boundary (ignoring positions outside
// the domain) form the outer / inner interface layers; the parent keeps its nodes
// up to fine distance 2 inside the child region, those at distance 2 being the ring
// rebuilt from co-located child nodes (twin nodes x_t,cf); outer-layer child nodes
// on parent positions are the twins x_t,fc; the other interface nodes are the
// reconstruction nodes x_r.  Distances are computed per brick from windowed
// membership bitmaps and 3-D prefix sums.
//
// Schedule (Sec. III.C, recursive over levels): one coarse step is 2^(L-1) ticks of
// the finest level; level l arrives every 2^(L-1-l) ticks.  At a tick, every arriving
// level stream-collides its bulk nodes (pull from its previous post-collision
// buffer); a level whose parent does not arrive is at its first substep and also
// collides its inner interface layer (the outer layer is skipped, step 1).  For each
// arriving parent/child pair the post-stream states of coarse-aligned points are
// gathered, then the child interface layers are reconstructed (steps 3-4) and the
// parent ring coalesced, and those nodes collide (step 5).  Everything reads the
// previous buffers and writes the next ones, so the bulk and coupling launches of a
// tick are independent and run as parallel graph branches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <condition_variable>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/elbm.h"
#include "elbm_dev.hpp"
#include "indicator.hpp"
#include "remesh.hpp"

using namespace elbm;

namespace {

struct Box {
  int64_t lo[3], hi[3];
};
struct SolidSpec {
  int64_t lo[3], n[3];
  std::vector<uint8_t> mask;
};

struct Level {
  std::vector<Box> boxes;
  std::vector<SolidSpec> solids;
  int64_t blo[3] = {0, 0, 0}, bn[3] = {1, 1, 1};
  int full[3] = {0, 0, 0};
  int64_t gdim[3] = {1, 1, 1};
  std::vector<int32_t> bgrid;  // brick grid -> brick id
  std::vector<int32_t> borg;   // [nb*3] brick origin relative to blo
  int32_t nb = 0;
  std::vector<uint8_t> cls;
  std::vector<uint32_t> mask;
  std::vector<float> weight;
  std::vector<int32_t> nbr;
  std::vector<uint8_t> exists, pd, ring, solid;
  double beta = 1.0;
  int64_t n_nodes = 0, n_fluid = 0, n_update = 0;
  std::vector<WorkItem> items1, items2;
  bool any_drag = false;
  size_t o_pop[2] = {0, 0}, o_cls = 0, o_mask = 0, o_w = 0, o_nbr = 0, o_force = 0, o_gamma = 0, o_drag = 0,
         o_borg = 0;
  bool force_on = false;
};

struct Pair {
  std::vector<GPoint> pts;
  std::vector<CItem> items;  // fine interface items (kind 0), stencils in global slots
  std::vector<CItem> ring;   // coarse ring items (kind 1)
  std::vector<CTile> tiles;  // item0 / pt0 relative to this pair's arrays
  std::vector<int32_t> tile_rows;
  std::vector<CItem> titems;  // fine items in tile order, stencils in tile rows
  std::vector<StencilEntry> tsten;
  double fac_pc = 1, fac_cp = 1;
};

struct Tick {
  int lmin;
  size_t sc_off, sc_n, gp_off, gp_n, tile_off, tile_n, ring_off, ring_n;
  size_t sc_plain;  // the last sc_plain items of the tick are plain bricks
  // XCD tables (xcd_remap 1): item of each dispatch position for the whole tick, for its
  // special bricks and for its plain bricks (offsets into perm_all)
  size_t pu_off, ps_off, pp_off;
};

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace

struct elbm_ctx {
  int D = 3, Q = 27, L = 1, storage = ST_F32;
  int64_t N[3] = {1, 1, 1};
  int periodic[3] = {0, 0, 0};
  double nu0 = 0;
  int face_kind[6] = {0, 0, 0, 0, 0, 0};
  double face_u[6][3] = {};
  double Fu[3] = {0, 0, 0};
  Level lev[MAXL];
  std::vector<Pair> pairs;
  std::vector<Tick> ticks;
  std::vector<WorkItem> sc_all, red_items;
  std::vector<int32_t> perm_all;
  std::vector<GPoint> gp_all;
  std::vector<CItem> fine_all, ring_all;
  std::vector<CTile> tiles_all;
  std::vector<int32_t> tile_rows_all;
  std::vector<StencilEntry> sten, tsten_all;
  int lds_rows = 1, lds_ents = 1, lds_items = 1;
  int stage_cols = 0;
  bool finalized = false, bound = false;
  std::string err;
  // workspace layout
  size_t ws_need = 0, o_levstatic = 0, o_pairstatic = 0, o_sc = 0, o_perm = 0, o_gp = 0, o_fine = 0, o_ring = 0, o_tiles = 0,
         o_trows = 0, o_sten = 0, o_stage = 0, o_redit = 0, o_part = 0, o_res = 0, o_tmp = 0;
  size_t tmp_bytes = 0;
  char *ws = nullptr;
  hipStream_t stream = nullptr, side = nullptr, cap = nullptr, side2 = nullptr;
  hipEvent_t ev_fork[64], ev_join[64], ev_fork2[64], ev_join2[64];
  int n_events = 0;
  hipGraphExec_t graph[2] = {nullptr, nullptr};   // one coarse step, by level-0 parity
  hipGraphExec_t graphm[2] = {nullptr, nullptr};  // use_graph coarse steps, by level-0 parity
  bool graph_valid = false;
  int parity = 0;  // buffer index of level 0
  int64_t drag_steps[MAXL] = {};
  // launch config
  int use_graph = 1, wg_per_cu = 0, xcd_remap = 1, threads = 256, occ = 1, pipe = 0;
  bool gamma_on = false;
  bool timing = false;
  std::vector<hipEvent_t> tev;
  std::vector<std::pair<size_t, size_t>> pair_gp;  // interpolation points of each pair (offset, count)
  // discrete adjoint
  struct Adjoint {
    bool bound = false, pending = false;
    char *ws = nullptr;
    int nmax = 0, K = 1;
    // two tapes (and two staged-row tapes): the recomputation of one segment fills one
    // while the reverse sweep of the next segment reads the other
    size_t o_tape[2][MAXL] = {}, o_ckpt = 0, o_lam[MAXL][2] = {}, o_lg[MAXL][2] = {}, o_lF[MAXL] = {},
           o_amask[MAXL] = {}, o_alev = 0, o_astage = 0, o_tofs = 0, o_tsten = 0, o_items = 0, o_part = 0,
           o_res = 0, o_stape[2] = {}, o_bitems = 0, need = 0;
    int rset = 0;  // tape set the reverse sweep reads
    // staged rows of every coupling tick of a segment, kept from the recomputation for
    // the reverse sweep: slot of tick t (-1 without coupling), slots per coarse step,
    // bytes per slot
    std::vector<int> ctick;
    int nct = 0;
    size_t stage_bytes = 0;
    bool has_amask[MAXL] = {};
    std::vector<WorkItem> items;                  // every brick of the arriving levels, per tick
    std::vector<std::pair<size_t, size_t>> tick;  // (offset, count) into items per tick
    // fused launches: after reversing tick t, the streaming transpose of t together with
    // the collision adjoint of the tick before it (t - 1, or T of the previous coarse
    // step): the bricks of the levels of either tick, thr of the colliding tick
    std::vector<WorkItem> bitems;
    std::vector<std::pair<size_t, size_t>> btick;
    std::vector<int32_t> tofs;
    std::vector<StencilEntry> tsten;
    std::vector<uint32_t> amask[MAXL];
    int cur[MAXL] = {};  // lam buffer holding the adjoint of the current state
    int lgc[MAXL] = {};  // lg buffer holding the level's latest collision adjoint
    int n = 0, objective = 0, body_level = -1;
    double dir[3] = {0, 0, 0}, J = 0;
    float ms[4] = {0, 0, 0, 0};  // forward with checkpoints, recomputation, reverse sweep, whole backward pass
  } adj;
  int cu_count = 256;
  void *static_staging = nullptr;  // this device's copy of the static staging buffer
};

#define FAIL(ctx, code, ...)                                          \
  do {                                                                \
    char _b[512];                                                     \
    snprintf(_b, sizeof(_b), __VA_ARGS__);                            \
    (ctx)->err = _b;                                                  \
    return code;                                                      \
  } while (0)

#define HIPCK(ctx, call)                                                          \
  do {                                                                            \
    hipError_t _e = (call);                                                       \
    if (_e != hipSuccess) FAIL(ctx, ELBM_EDEVICE, "%s: %s", #call, hipGetErrorString(_e)); \
  } while (0)

#define LCK(ctx, call)                                                                          \
  do {                                                                                          \
    int _e = (call);                                                                            \
    if (_e) FAIL(ctx, ELBM_EDEVICE, "%s: %s", #call, hipGetErrorString((hipError_t)_e));       \
  } while (0)

// Staging buffer of elbm_init_fields_static, for callers that cannot allocate device
// memory.  Each GPU the library runs on holds its own copy until the process ends.  In
// host code this name only stands for the symbol: its device address (per device) comes
// from hipGetSymbolAddress, taken once per device when a context binds.
constexpr size_t kStaticStagingBytes = (size_t)32 << 20;
static __device__ __align__(256) char scratch[kStaticStagingBytes];

namespace {

std::mutex g_staging_mu;
constexpr int kMaxDevices = 64;
void *g_staging_ptr[kMaxDevices] = {};

// device address of the static staging buffer on the current device (looked up once)
hipError_t static_staging_address(int dev, void **out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_staging_mu);
  if (!g_staging_ptr[dev]) {
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_staging_ptr[dev] = p;
  }
  *out = g_staging_ptr[dev];
  return hipSuccess;
}

// ------------------------------------------------------------------ geometry helpers
int64_t period(const elbm_ctx *c, int l, int a) { return c->N[a] << l; }
int64_t extent(const elbm_ctx *c, int l, int a) {
  if (a >= c->D) return 1;
  return c->periodic[a] ? (c->N[a] << l) : ((c->N[a] - 1) << l) + 1;
}
int64_t pmod(int64_t x, int64_t p) {
  int64_t r = x % p;
  return r < 0 ? r + p : r;
}
// canonical position (periodic wrap); false if outside a non-periodic axis
bool to_domain(const elbm_ctx *c, int l, int64_t x[3]) {
  for (int a = 0; a < 3; ++a) {
    if (a >= c->D) {
      if (x[a] != 0) return false;
      continue;
    }
    if (c->periodic[a]) x[a] = pmod(x[a], period(c, l, a));
    else if (x[a] < 0 || x[a] >= extent(c, l, a)) return false;
  }
  return true;
}
bool box_spans(const elbm_ctx *c, int l, const Box &b, int a) {
  return c->periodic[a] && b.hi[a] - b.lo[a] >= period(c, l, a) - 1;
}
// canonical in-domain x inside the union of level-l blocks (level 0: everywhere)
bool in_blocks(const elbm_ctx *c, int l, const int64_t x[3]) {
  if (l == 0) return true;
  for (const Box &b : c->lev[l].boxes) {
    bool in = true;
    for (int a = 0; a < c->D && in; ++a) {
      if (c->periodic[a]) {
        if (box_spans(c, l, b, a)) continue;
        in = pmod(x[a] - b.lo[a], period(c, l, a)) <= b.hi[a] - b.lo[a];
      } else {
        in = x[a] >= b.lo[a] && x[a] <= b.hi[a];
      }
    }
    if (in) return true;
  }
  return false;
}
// member: in the domain and in the level region
bool member(const elbm_ctx *c, int l, const int64_t xin[3]) {
  int64_t x[3] = {xin[0], xin[1], xin[2]};
  return to_domain(c, l, x) && in_blocks(c, l, x);
}
// "bad" position for distance purposes: in the domain but outside the region
bool bad_pos(const elbm_ctx *c, int l, const int64_t xin[3]) {
  int64_t x[3] = {xin[0], xin[1], xin[2]};
  if (!to_domain(c, l, x)) return false;
  return !in_blocks(c, l, x);
}
// direct distance (capped at 3) of a member position; -1 if not a member
int dist_direct(const elbm_ctx *c, int l, const int64_t x[3]) {
  if (!member(c, l, x)) return -1;
  if (l == 0) return 3;
  int k;
  for (k = 1; k <= 3; ++k) {
    const int kz = c->D == 3 ? k : 0;
    for (int64_t dz = -kz; dz <= kz; ++dz)
      for (int64_t dy = -k; dy <= k; ++dy)
        for (int64_t dx = -k; dx <= k; ++dx) {
          if (std::max(std::max(std::llabs(dx), std::llabs(dy)), std::llabs(dz)) != k) continue;
          int64_t y[3] = {x[0] + dx, x[1] + dy, x[2] + dz};
          if (bad_pos(c, l, y)) return k - 1;
        }
  }
  return 3;
}

// Windowed prefix sums of "bad" positions: counts over boxes in O(1).
struct Window {
  int64_t lo[3], n[3];
  std::vector<int32_t> S;  // (n+1)^3 inclusive prefix
  void build(const elbm_ctx *c, int l, const int64_t wlo[3], const int64_t whi[3]) {
    for (int a = 0; a < 3; ++a) {
      lo[a] = wlo[a];
      n[a] = whi[a] - wlo[a] + 1;
    }
    S.assign((size_t)(n[0] + 1) * (n[1] + 1) * (n[2] + 1), 0);
    auto at = [&](int64_t i, int64_t j, int64_t k) -> int32_t & {
      return S[(size_t)i + (size_t)(n[0] + 1) * ((size_t)j + (size_t)(n[1] + 1) * (size_t)k)];
    };
    for (int64_t k = 1; k <= n[2]; ++k)
      for (int64_t j = 1; j <= n[1]; ++j)
        for (int64_t i = 1; i <= n[0]; ++i) {
          int64_t p[3] = {lo[0] + i - 1, lo[1] + j - 1, lo[2] + k - 1};
          int32_t v = l == 0 ? 0 : (int32_t)bad_pos(c, l, p);
          at(i, j, k) = v + at(i - 1, j, k) + at(i, j - 1, k) + at(i, j, k - 1) - at(i - 1, j - 1, k) -
                        at(i - 1, j, k - 1) - at(i, j - 1, k - 1) + at(i - 1, j - 1, k - 1);
        }
  }
  int32_t count(const int64_t a[3], const int64_t b[3]) const {  // inclusive, must lie in the window
    int64_t i0 = a[0] - lo[0], j0 = a[1] - lo[1], k0 = a[2] - lo[2];
    int64_t i1 = b[0] - lo[0] + 1, j1 = b[1] - lo[1] + 1, k1 = b[2] - lo[2] + 1;
    auto at = [&](int64_t i, int64_t j, int64_t k) -> int32_t {
      return S[(size_t)i + (size_t)(n[0] + 1) * ((size_t)j + (size_t)(n[1] + 1) * (size_t)k)];
    };
    return at(i1, j1, k1) - at(i0, j1, k1) - at(i1, j0, k1) - at(i1, j1, k0) + at(i0, j0, k1) + at(i0, j1, k0) +
           at(i1, j0, k0) - at(i0, j0, k0);
  }
  // distance capped at 3 for a member position (caller checks membership)
  int dist(int D, const int64_t x[3]) const {
    for (int k = 1; k <= 3; ++k) {
      int64_t a[3] = {x[0] - k, x[1] - k, D == 3 ? x[2] - k : x[2]};
      int64_t b[3] = {x[0] + k, x[1] + k, D == 3 ? x[2] + k : x[2]};
      if (count(a, b)) return k - 1;
    }
    return 3;
  }
};

template <int D> struct BK {
  static constexpr int X = Brick<D>::BX, Y = Brick<D>::BY, Z = Brick<D>::BZ;
};
int bdim(int D, int a) {
  if (D == 2) return a == 0 ? Brick<2>::BX : (a == 1 ? Brick<2>::BY : 1);
  return a == 0 ? Brick<3>::BX : (a == 1 ? Brick<3>::BY : Brick<3>::BZ);
}

int vel(int D, int i, int a) {
  if (a == 0) return i % 3 - 1;
  if (a == 1) return (i / 3) % 3 - 1;
  return D == 3 ? i / 9 - 1 : 0;
}
double wgt(int D, int i) {
  double w = 1;
  for (int a = 0; a < D; ++a) w *= vel(D, i, a) == 0 ? 2.0 / 3.0 : 1.0 / 6.0;
  return w;
}

// equilibrium minus weights at (rho=1, u), host double (inlet populations)
void heq_host(int D, const double u[3], double *h) {
  const int Q = D == 2 ? 9 : 27;
  double a[3][3];
  for (int ax = 0; ax < 3; ++ax) {
    double t = 3 * u[ax] * u[ax], sig = t / (1 + std::sqrt(1 + t));
    a[ax][0] = 2 * sig - 3 * u[ax];
    a[ax][1] = -sig;
    a[ax][2] = 2 * sig + 3 * u[ax];
  }
  for (int i = 0; i < Q; ++i) {
    double p = 1;
    for (int ax = 0; ax < D; ++ax) p *= 1 + a[ax][vel(D, i, ax) + 1];
    h[i] = wgt(D, i) * (p - 1);
  }
}

struct NodeRef {
  int32_t brick = -1;
  int32_t node = 0;
};

NodeRef locate(const elbm_ctx *c, int l, const int64_t xin[3]) {
  NodeRef r;
  int64_t x[3] = {xin[0], xin[1], xin[2]};
  if (!to_domain(c, l, x)) return r;
  const Level &L = c->lev[l];
  int64_t g[3], loc[3];
  for (int a = 0; a < 3; ++a) {
    int64_t p = x[a] - L.blo[a];
    if (p < 0 || p >= L.bn[a]) return r;
    g[a] = p / bdim(c->D, a);
    loc[a] = p % bdim(c->D, a);
  }
  int32_t b = L.bgrid[(size_t)g[0] + (size_t)L.gdim[0] * ((size_t)g[1] + (size_t)L.gdim[1] * (size_t)g[2])];
  if (b < 0) return r;
  int32_t n = (int32_t)(loc[0] + bdim(c->D, 0) * (loc[1] + bdim(c->D, 1) * loc[2]));
  if (!L.exists[(size_t)b * BN + n]) return r;
  r.brick = b;
  r.node = n;
  return r;
}

elbm_status build_level_geometry(elbm_ctx *c, int l);
elbm_status build_level_links(elbm_ctx *c, int l);
elbm_status build_pairs(elbm_ctx *c);
void build_schedule(elbm_ctx *c);
void build_layout(elbm_ctx *c);

elbm_status build_level_geometry(elbm_ctx *c, int l) {
  Level &L = c->lev[l];
  const int D = c->D;
  // index box
  for (int a = 0; a < 3; ++a) {
    L.full[a] = 0;
    if (a >= D) {
      L.blo[a] = 0;
      L.bn[a] = 1;
      continue;
    }
    if (l == 0) {
      L.blo[a] = 0;
      L.bn[a] = extent(c, 0, a);
      L.full[a] = c->periodic[a];
      continue;
    }
    bool whole = false;
    int64_t mn = INT64_MAX, mx = INT64_MIN;
    for (const Box &b : L.boxes) {
      if (c->periodic[a] && (box_spans(c, l, b, a) || b.hi[a] >= period(c, l, a))) whole = true;
      mn = std::min(mn, b.lo[a]);
      mx = std::max(mx, b.hi[a]);
    }
    if (whole) {
      L.blo[a] = 0;
      L.bn[a] = period(c, l, a);
      L.full[a] = 1;
    } else {
      L.blo[a] = mn;
      L.bn[a] = mx - mn + 1;
    }
  }
  for (int a = 0; a < D; ++a) {
    if (L.full[a] && L.bn[a] % bdim(D, a))
      FAIL(c, ELBM_EINVAL, "level %d: periodic axis %d has %lld nodes, not a multiple of the brick size %d", l, a,
           (long long)L.bn[a], bdim(D, a));
  }
  for (int a = 0; a < 3; ++a) L.gdim[a] = (L.bn[a] + bdim(D, a) - 1) / bdim(D, a);
  const size_t ng = (size_t)L.gdim[0] * L.gdim[1] * L.gdim[2];
  // candidate bricks
  std::vector<uint8_t> cand(ng, l == 0 ? 1 : 0);
  if (l > 0) {
    for (const Box &b : L.boxes) {
      // per axis, list of index-box coordinate ranges covered by the box
      std::vector<std::pair<int64_t, int64_t>> rng[3];
      for (int a = 0; a < 3; ++a) {
        if (a >= D) {
          rng[a].push_back({0, 0});
          continue;
        }
        if (c->periodic[a] && box_spans(c, l, b, a)) {
          rng[a].push_back({0, L.bn[a] - 1});
        } else if (c->periodic[a] && L.full[a]) {
          int64_t P = period(c, l, a);
          int64_t lo = b.lo[a], hi = b.hi[a];
          if (hi < P) rng[a].push_back({lo, hi});
          else {
            rng[a].push_back({lo, P - 1});
            rng[a].push_back({0, hi - P});
          }
        } else {
          rng[a].push_back({b.lo[a] - L.blo[a], b.hi[a] - L.blo[a]});
        }
      }
      for (auto rx : rng[0])
        for (auto ry : rng[1])
          for (auto rz : rng[2])
            for (int64_t gz = rz.first / bdim(D, 2); gz <= rz.second / bdim(D, 2); ++gz)
              for (int64_t gy = ry.first / bdim(D, 1); gy <= ry.second / bdim(D, 1); ++gy)
                for (int64_t gx = rx.first / bdim(D, 0); gx <= rx.second / bdim(D, 0); ++gx)
                  cand[(size_t)gx + L.gdim[0] * ((size_t)gy + L.gdim[1] * (size_t)gz)] = 1;
    }
  }
  // bounding box of the child level's blocks (level l+1 coordinates) to skip work
  const bool has_child = l + 1 < c->L;
  L.bgrid.assign(ng, -1);
  L.borg.clear();
  L.exists.clear();
  L.pd.clear();
  L.ring.clear();
  L.weight.clear();
  L.nb = 0;
  std::vector<uint8_t> ex(BN), pdv(BN), rg(BN);
  std::vector<float> wv(BN);
  const double base = std::ldexp(1.0, -l * D);
  for (int64_t gz = 0; gz < L.gdim[2]; ++gz)
    for (int64_t gy = 0; gy < L.gdim[1]; ++gy)
      for (int64_t gx = 0; gx < L.gdim[0]; ++gx) {
        const size_t gi = (size_t)gx + L.gdim[0] * ((size_t)gy + L.gdim[1] * (size_t)gz);
        if (!cand[gi]) continue;
        int64_t o[3] = {gx * bdim(D, 0), gy * bdim(D, 1), gz * bdim(D, 2)};
        int64_t x0[3], x1[3];  // level coordinates of the brick
        for (int a = 0; a < 3; ++a) {
          x0[a] = L.blo[a] + o[a];
          x1[a] = x0[a] + bdim(D, a) - 1;
        }
        Window wa, wb;
        int64_t m = 3;
        int64_t alo[3] = {x0[0] - m, x0[1] - m, D == 3 ? x0[2] - m : 0};
        int64_t ahi[3] = {x1[0] + m, x1[1] + m, D == 3 ? x1[2] + m : 0};
        if (l > 0) wa.build(c, l, alo, ahi);
        if (has_child) {
          int64_t blo2[3] = {2 * x0[0] - m, 2 * x0[1] - m, D == 3 ? 2 * x0[2] - m : 0};
          int64_t bhi2[3] = {2 * x1[0] + m, 2 * x1[1] + m, D == 3 ? 2 * x1[2] + m : 0};
          wb.build(c, l + 1, blo2, bhi2);
        }
        bool any = false;
        for (int n = 0; n < BN; ++n) {
          int64_t loc[3] = {n % bdim(D, 0), (n / bdim(D, 0)) % bdim(D, 1), n / (bdim(D, 0) * bdim(D, 1))};
          int64_t x[3] = {x0[0] + loc[0], x0[1] + loc[1], x0[2] + loc[2]};
          ex[n] = 0;
          pdv[n] = 0;
          rg[n] = 0;
          wv[n] = 0;
          if (loc[2] >= bdim(D, 2)) continue;
          bool inside = true;
          for (int a = 0; a < 3; ++a) inside = inside && (x[a] - L.blo[a] < L.bn[a]);
          if (!inside || !member(c, l, x)) continue;
          int dch = -1;
          if (has_child) {
            int64_t y[3] = {2 * x[0], 2 * x[1], 2 * x[2]};
            if (member(c, l + 1, y)) dch = wb.dist(D, y);
          }
          if (dch >= 3) continue;  // deep inside the child: no parent node (Sec. III)
          ex[n] = 1;
          any = true;
          rg[n] = dch == 2;
          int d = l > 0 ? wa.dist(D, x) : 3;
          pdv[n] = (uint8_t)d;
          // owned-volume weight: the child owns its region eroded by one fine spacing;
          // sub-cell sigma of x is owned iff the 4^D node block [x-1,x+2] / [x-2,x+1]
          // (per axis, by sign) contains no in-domain position outside the region
          double wt = base;
          if (rg[n]) wt = 0;
          else if (l > 0 && d < 2) {
            int cnt = 0, tot = 1 << D;
            for (int s = 0; s < tot; ++s) {
              int64_t a0[3] = {x[0], x[1], x[2]}, a1[3] = {x[0], x[1], x[2]};
              for (int a = 0; a < D; ++a) {
                bool plus = (s >> a) & 1;
                a0[a] = x[a] + (plus ? -1 : -2);
                a1[a] = x[a] + (plus ? 2 : 1);
              }
              cnt += wa.count(a0, a1) == 0;
            }
            wt = base * cnt / tot;
          }
          wv[n] = (float)wt;
        }
        if (!any) continue;
        const int32_t b = L.nb++;
        L.bgrid[gi] = b;
        L.borg.push_back((int32_t)o[0]);
        L.borg.push_back((int32_t)o[1]);
        L.borg.push_back((int32_t)o[2]);
        L.exists.insert(L.exists.end(), ex.begin(), ex.end());
        L.pd.insert(L.pd.end(), pdv.begin(), pdv.end());
        L.ring.insert(L.ring.end(), rg.begin(), rg.end());
        L.weight.insert(L.weight.end(), wv.begin(), wv.end());
      }
  L.solid.assign((size_t)L.nb * BN, 0);
  for (const SolidSpec &s : L.solids) {
    for (int64_t z = 0; z < s.n[2]; ++z)
      for (int64_t y = 0; y < s.n[1]; ++y)
        for (int64_t x = 0; x < s.n[0]; ++x) {
          if (!s.mask[(size_t)x + s.n[0] * ((size_t)y + s.n[1] * (size_t)z)]) continue;
          int64_t p[3] = {s.lo[0] + x, s.lo[1] + y, s.lo[2] + z};
          NodeRef r = locate(c, l, p);
          if (r.brick < 0)
            FAIL(c, ELBM_EINVAL, "level %d: solid node (%lld,%lld,%lld) is not a node of this level", l,
                 (long long)p[0], (long long)p[1], (long long)p[2]);
          size_t k = (size_t)r.brick * BN + r.node;
          if (L.pd[k] < 2 || L.ring[k])
            FAIL(c, ELBM_EINVAL, "level %d: solid node (%lld,%lld,%lld) lies on an interface layer", l,
                 (long long)p[0], (long long)p[1], (long long)p[2]);
          L.solid[k] = 1;
          L.weight[k] = 0;
        }
  }
  L.beta = 1.0 / (6.0 * c->nu0 * std::ldexp(1.0, l) + 1.0);  // Eq. visc with nu_l = 2^l nu0
  return ELBM_OK;
}

elbm_status build_level_links(elbm_ctx *c, int l) {
  Level &L = c->lev[l];
  const int D = c->D, Q = c->Q;
  L.cls.assign((size_t)L.nb * BN, 0);
  L.mask.assign((size_t)L.nb * BN, 0);
  L.n_nodes = L.n_fluid = L.n_update = 0;
  L.any_drag = false;
  L.items1.clear();
  L.items2.clear();
  for (int32_t b = 0; b < L.nb; ++b) {
    bool m1 = false, m2 = false, dr = false;
    for (int n = 0; n < BN; ++n) {
      const size_t k = (size_t)b * BN + n;
      if (!L.exists[k]) continue;
      L.n_nodes++;
      if (L.solid[k]) continue;
      L.n_fluid++;
      int64_t x[3];
      int64_t loc[3] = {n % bdim(D, 0), (n / bdim(D, 0)) % bdim(D, 1), n / (bdim(D, 0) * bdim(D, 1))};
      for (int a = 0; a < 3; ++a) x[a] = L.blo[a] + L.borg[3 * b + a] + loc[a];
      int mode = 2;
      if (L.ring[k] || L.pd[k] == 0) mode = 0;
      else if (L.pd[k] == 1) mode = 1;
      uint32_t bb = 0, inl = 0, outm = 0, solidlinks = 0, walllinks = 0;
      for (int i = 0; i < Q; ++i) {
        int64_t y[3];
        for (int a = 0; a < 3; ++a) y[a] = x[a] - vel(D, i, a);
        int kind = 0;  // 0 node, 1 wall, 2 inlet, 3 outflow
        for (int a = 0; a < D; ++a) {
          if (c->periodic[a]) continue;
          int face = -1;
          if (y[a] < 0) face = 2 * a;
          else if (y[a] > extent(c, l, a) - 1) face = 2 * a + 1;
          if (face < 0) continue;
          int fk = c->face_kind[face];
          if (fk == ELBM_FACE_WALL) kind = 1;
          else if (fk == ELBM_FACE_INLET && kind != 1) kind = 2;
          else if (fk == ELBM_FACE_OUTFLOW) {
            if (kind == 0) kind = 3;
            y[a] += (face & 1) ? -1 : 1;
          }
        }
        if (kind == 1) {
          bb |= 1u << i;
          walllinks |= 1u << i;
          continue;
        }
        if (kind == 2) {
          inl |= 1u << i;
          continue;
        }
        if (kind == 3) outm |= 1u << i;
        NodeRef r = locate(c, l, y);
        if (r.brick >= 0 && L.solid[(size_t)r.brick * BN + r.node]) {
          if (kind == 3)
            FAIL(c, ELBM_EINVAL, "level %d: outflow source is solid at (%lld,%lld,%lld)", l, (long long)x[0],
                 (long long)x[1], (long long)x[2]);
          bb |= 1u << i;
          solidlinks |= 1u << i;
          continue;
        }
        if (mode > 0 && r.brick < 0)
          FAIL(c, ELBM_EINVAL,
               "level %d: node (%lld,%lld,%lld) pulls population %d from a position with no node (nesting margin "
               "or interface alignment violated)",
               l, (long long)x[0], (long long)x[1], (long long)x[2], i);
      }
      const int kinds = (bb != 0) + (inl != 0) + (outm != 0);
      if (kinds > 1)
        FAIL(c, ELBM_EINVAL, "level %d: node (%lld,%lld,%lld) mixes wall/solid, inlet and outflow links", l,
             (long long)x[0], (long long)x[1], (long long)x[2]);
      if (solidlinks && walllinks)
        FAIL(c, ELBM_EINVAL, "level %d: node (%lld,%lld,%lld) touches both a wall and a solid", l,
             (long long)x[0], (long long)x[1], (long long)x[2]);
      if (mode == 0 && kinds)
        FAIL(c, ELBM_EINVAL, "level %d: interface node (%lld,%lld,%lld) touches a boundary", l, (long long)x[0],
             (long long)x[1], (long long)x[2]);
      uint8_t cl = (uint8_t)mode | CLS_FLUID;
      if (bb) cl |= CLS_LINKS;
      if (inl) cl |= CLS_INLET;
      if (outm) cl |= CLS_OUTFLOW;
      if (solidlinks) {
        cl |= CLS_DRAG;
        dr = true;
      }
      L.cls[k] = cl;
      L.mask[k] = bb | inl | outm;
      if (mode >= 1) m1 = true;
      if (mode == 2) m2 = true;
      if (mode > 0 || L.ring[k] || L.pd[k] <= 1) L.n_update++;
    }
    // plain bricks: every node fluid, stream-collided at this threshold, plain links only
    bool plain1 = true, plain2 = true, links = false;
    for (int n = 0; n < BN; ++n) {
      const uint8_t cl = L.cls[(size_t)b * BN + n];
      const bool ok = (cl & CLS_FLUID) && !(cl & (CLS_LINKS | CLS_INLET | CLS_OUTFLOW | CLS_DRAG));
      plain1 = plain1 && ok && (cl & CLS_MODE) >= 1;
      plain2 = plain2 && ok && (cl & CLS_MODE) >= 2;
      links = links || (cl & (CLS_LINKS | CLS_INLET | CLS_OUTFLOW));
    }
    WorkItem w;
    w.brick = b;
    w.level = (uint8_t)l;
    w.drag = dr;
    w.flags = 0;
    if (m1) {
      w.thr = 1;
      w.flags = (uint8_t)((plain1 ? WI_PLAIN : 0) | (links ? WI_LINKS : 0));
      L.items1.push_back(w);
    }
    if (m2) {
      w.thr = 2;
      w.flags = (uint8_t)((plain2 ? WI_PLAIN : 0) | (links ? WI_LINKS : 0));
      L.items2.push_back(w);
    }
    L.any_drag = L.any_drag || dr;
  }
  // neighbour table (periodic wrap on whole-period axes)
  L.nbr.assign((size_t)L.nb * 27, -1);
  for (int32_t b = 0; b < L.nb; ++b) {
    int64_t g[3] = {L.borg[3 * b] / bdim(D, 0), L.borg[3 * b + 1] / bdim(D, 1), L.borg[3 * b + 2] / bdim(D, 2)};
    for (int k = 0; k < 27; ++k) {
      int64_t q[3] = {g[0] + k % 3 - 1, g[1] + (k / 3) % 3 - 1, g[2] + k / 9 - 1};
      bool ok = true;
      for (int a = 0; a < 3; ++a) {
        if (q[a] < 0 || q[a] >= L.gdim[a]) {
          if (L.full[a] && a < D) q[a] = pmod(q[a], L.gdim[a]);
          else ok = false;
        }
      }
      if (!ok) continue;
      L.nbr[(size_t)b * 27 + k] = L.bgrid[(size_t)q[0] + L.gdim[0] * ((size_t)q[1] + L.gdim[1] * (size_t)q[2])];
    }
  }
  return ELBM_OK;
}

bool plain_bulk(const elbm_ctx *c, int l, NodeRef r) {
  if (r.brick < 0) return false;
  const Level &L = c->lev[l];
  const size_t k = (size_t)r.brick * BN + r.node;
  const uint8_t cl = L.cls[k];
  return (cl & CLS_FLUID) && (cl & CLS_MODE) == 2 && !(cl & (CLS_LINKS | CLS_INLET | CLS_OUTFLOW)) && !L.ring[k];
}

elbm_status build_pairs(elbm_ctx *c) {
  const int D = c->D;
  c->pairs.assign(c->L > 1 ? c->L - 1 : 0, Pair());
  c->sten.clear();
  int slots = 0;
  for (int p = 0; p + 1 < c->L; ++p) {
    Pair &P = c->pairs[p];
    const Level &Lp = c->lev[p], &Lc = c->lev[p + 1];
    P.fac_pc = Lp.beta / (2.0 * Lc.beta);  // Eq. f_neq_rescaling_iso with r = 2
    P.fac_cp = 2.0 * Lc.beta / Lp.beta;
    std::unordered_map<uint64_t, int32_t> slot_of;
    // slot of each coarse point already placed: a point is named by many stencils
    // (up to 64 per fine node), and it always maps to the same node
    std::unordered_map<uint64_t, int32_t> slot_at;
    auto point = [&](const int64_t X[3], int32_t &slot) -> elbm_status {
      const uint64_t xkey = ((uint64_t)(X[0] & 0x1fffff) << 42) | ((uint64_t)(X[1] & 0x1fffff) << 21) |
                            (uint64_t)(X[2] & 0x1fffff);
      auto hit = slot_at.find(xkey);
      if (hit != slot_at.end()) {
        slot = hit->second;
        return ELBM_OK;
      }
      int64_t xc[3] = {2 * X[0], 2 * X[1], 2 * X[2]};
      int lvl;
      NodeRef r;
      int dch = member(c, p + 1, xc) ? dist_direct(c, p + 1, xc) : -1;
      if (dch >= 2) {
        lvl = p + 1;
        r = locate(c, p + 1, xc);
      } else {
        lvl = p;
        r = locate(c, p, X);
      }
      if (!plain_bulk(c, lvl, r))
        FAIL(c, ELBM_EINVAL,
             "interface %d/%d: interpolation point (%lld,%lld,%lld) has no plain bulk node on level %d (nesting "
             "margin too small or boundary too close)",
             p, p + 1, (long long)X[0], (long long)X[1], (long long)X[2], lvl);
      uint64_t key = ((uint64_t)lvl << 56) ^ ((uint64_t)r.brick << 16) ^ (uint64_t)r.node;
      auto it = slot_of.find(key);
      if (it != slot_of.end()) {
        slot = it->second;
        slot_at[xkey] = slot;
        return ELBM_OK;
      }
      GPoint g;
      g.brick = r.brick;
      g.node = (uint16_t)r.node;
      g.level = (uint8_t)lvl;
      g.pair = (uint8_t)p;
      g.slot = slots++;
      P.pts.push_back(g);
      slot_of[key] = g.slot;
      slot_at[xkey] = g.slot;
      slot = g.slot;
      return ELBM_OK;
    };
    static const float w4[4] = {-1.0f / 16, 9.0f / 16, 9.0f / 16, -1.0f / 16};
    // fine interface layers
    for (int32_t b = 0; b < Lc.nb; ++b)
      for (int n = 0; n < BN; ++n) {
        const size_t k = (size_t)b * BN + n;
        if (!Lc.exists[k] || Lc.solid[k] || Lc.pd[k] > 1) continue;
        int64_t loc[3] = {n % bdim(D, 0), (n / bdim(D, 0)) % bdim(D, 1), n / (bdim(D, 0) * bdim(D, 1))};
        int64_t x[3];
        for (int a = 0; a < 3; ++a) x[a] = Lc.blo[a] + Lc.borg[3 * b + a] + loc[a];
        int64_t xw[3] = {x[0], x[1], x[2]};
        to_domain(c, p + 1, xw);
        int npt[3] = {1, 1, 1};
        int64_t pts[3][4];
        float wts[3][4];
        for (int a = 0; a < 3; ++a) {
          if (a < D && (xw[a] & 1)) {
            npt[a] = 4;
            for (int q = 0; q < 4; ++q) {
              pts[a][q] = (xw[a] - 3 + 2 * q) / 2;
              wts[a][q] = w4[q];
            }
          } else {
            pts[a][0] = xw[a] / 2;
            wts[a][0] = 1.0f;
          }
        }
        CItem it;
        it.brick = b;
        it.node = (uint16_t)n;
        it.level = (uint8_t)(p + 1);
        it.kind = 0;
        it.a = (int32_t)c->sten.size();
        it.b = npt[0] * npt[1] * npt[2];
        for (int qz = 0; qz < npt[2]; ++qz)
          for (int qy = 0; qy < npt[1]; ++qy)
            for (int qx = 0; qx < npt[0]; ++qx) {
              int64_t X[3] = {pts[0][qx], pts[1][qy], pts[2][qz]};
              int32_t slot;
              elbm_status s = point(X, slot);
              if (s) return s;
              StencilEntry e;
              e.slot = slot;
              e.w = wts[0][qx] * wts[1][qy] * wts[2][qz];
              c->sten.push_back(e);
            }
        P.items.push_back(it);
      }
    // tiles: fine interface nodes of one brick, longest stencils first (uniform loop
    // counts within a wavefront), split when the distinct rows exceed the LDS budget
    {
      const int maxr = couple_max_rows(D, c->storage), maxe = couple_max_entries();
      std::vector<CItem> its = P.items;
      std::stable_sort(its.begin(), its.end(), [](const CItem &x, const CItem &y) {
        return x.brick != y.brick ? x.brick < y.brick : x.b > y.b;
      });
      size_t k = 0;
      while (k < its.size()) {
        const int32_t br = its[k].brick;
        CTile t;
        t.item0 = (int32_t)P.titems.size();
        t.pt0 = (int32_t)P.tile_rows.size();
        t.nitem = 0;
        t.npt = 0;
        t.e0 = (int32_t)P.tsten.size();
        t.ne = 0;
        std::unordered_map<int32_t, int32_t> local;
        while (k < its.size() && its[k].brick == br) {
          const CItem &it = its[k];
          int add = 0;
          for (int e = it.a; e < it.a + it.b; ++e) add += local.count(c->sten[e].slot) ? 0 : 1;
          // close the tile (the same brick continues) when its rows, entries or nodes
          // (whose sums reuse the row area) exceed LDS
          if ((t.npt + add > maxr || t.ne + it.b > maxe || t.nitem + 1 > maxr) && t.nitem > 0) break;
          t.ne += it.b;
          CItem ti = it;
          ti.a = (int32_t)P.tsten.size();
          for (int e = it.a; e < it.a + it.b; ++e) {
            auto f = local.find(c->sten[e].slot);
            int32_t li;
            if (f == local.end()) {
              li = t.npt++;
              local[c->sten[e].slot] = li;
              P.tile_rows.push_back(c->sten[e].slot);
            } else {
              li = f->second;
            }
            StencilEntry se;
            se.slot = li;
            se.w = c->sten[e].w;
            P.tsten.push_back(se);
          }
          P.titems.push_back(ti);
          t.nitem++;
          ++k;
        }
        c->lds_rows = std::max(c->lds_rows, (int)t.npt);
        c->lds_ents = std::max(c->lds_ents, (int)t.ne);
        c->lds_items = std::max(c->lds_items, (int)t.nitem);
        P.tiles.push_back(t);
      }
    }
    // parent ring
    for (int32_t b = 0; b < Lp.nb; ++b)
      for (int n = 0; n < BN; ++n) {
        const size_t k = (size_t)b * BN + n;
        if (!Lp.exists[k] || !Lp.ring[k]) continue;
        int64_t loc[3] = {n % bdim(D, 0), (n / bdim(D, 0)) % bdim(D, 1), n / (bdim(D, 0) * bdim(D, 1))};
        int64_t x[3];
        for (int a = 0; a < 3; ++a) x[a] = Lp.blo[a] + Lp.borg[3 * b + a] + loc[a];
        int64_t xc[3] = {2 * x[0], 2 * x[1], 2 * x[2]};
        NodeRef r = locate(c, p + 1, xc);
        if (!plain_bulk(c, p + 1, r))
          FAIL(c, ELBM_EINVAL, "interface %d/%d: ring node (%lld,%lld,%lld) has no plain fine twin", p, p + 1,
               (long long)x[0], (long long)x[1], (long long)x[2]);
        if (Lp.cls[k] & (CLS_LINKS | CLS_INLET | CLS_OUTFLOW))
          FAIL(c, ELBM_EINVAL, "interface %d/%d: ring node touches a boundary", p, p + 1);
        CItem it;
        it.brick = b;
        it.node = (uint16_t)n;
        it.level = (uint8_t)p;
        it.kind = 1;
        it.a = r.brick;
        it.b = r.node;
        P.ring.push_back(it);
      }
  }
  c->stage_cols = slots;
  return ELBM_OK;
}

size_t store_bytes(int st);

// Whether gather + coupling is the longer of the two branches of a coupling tick, from
// rates measured on MI355X while both run: the stream-collide moves 3.8 TB/s of its
// bricks' populations (read + write, ~14.5 ns per 3-D FP32 brick); gather + coupling
// take ~10 us plus ~20 ns per coupling workgroup plus ~0.25 ns per interpolation
// point.  (Two-level channel, FP32: 82 us estimated against 58 us, measured 77 and
// 55 us; on the four-level forest's ticks the coupling branch is the longer one.)
// With 16-bit storage the stream-collide is bound by its arithmetic, not its bytes, and
// the coupling kernels share its SIMDs: there the coupling branch is the longer one in
// every coupling tick measured (the three-level sphere's level 0-2 tick: ~190 us of
// gather + coupling beside a 158 us stream-collide), so it is always captured first.
bool coupling_longer(const elbm_ctx *c, const Tick &tk) {
  if (tk.tile_n + tk.ring_n == 0) return false;
  if (store_bytes(c->storage) == 2) return true;
  const double sc_ns = (double)tk.sc_n * BN * c->Q * 2.0 * (double)store_bytes(c->storage) / 3800.0;
  const double cp_ns = 10000.0 + 20.0 * (double)(tk.tile_n + (tk.ring_n + 255) / 256) + 0.25 * (double)tk.gp_n;
  return cp_ns > sc_ns;
}

void build_schedule(elbm_ctx *c) {
  c->ticks.clear();
  c->sc_all.clear();
  c->perm_all.clear();
  c->gp_all.clear();
  c->fine_all.clear();
  c->ring_all.clear();
  c->tiles_all.clear();
  c->tile_rows_all.clear();
  c->tsten_all.clear();
  // pair lists laid out by parent level so that the pairs of a tick are contiguous
  std::vector<size_t> gp_start(c->L + 1, 0), tl_start(c->L + 1, 0), rg_start(c->L + 1, 0);
  for (int p = 0; p + 1 < c->L; ++p) {
    const Pair &P = c->pairs[p];
    gp_start[p] = c->gp_all.size();
    tl_start[p] = c->tiles_all.size();
    rg_start[p] = c->ring_all.size();
    c->gp_all.insert(c->gp_all.end(), P.pts.begin(), P.pts.end());
    const int32_t item_base = (int32_t)c->fine_all.size(), row_base = (int32_t)c->tile_rows_all.size();
    const int32_t sten_base = (int32_t)c->tsten_all.size();
    for (CTile t : P.tiles) {
      t.item0 += item_base;
      t.pt0 += row_base;
      t.e0 += sten_base;
      c->tiles_all.push_back(t);
    }
    for (CItem it : P.titems) {
      it.a += sten_base;
      c->fine_all.push_back(it);
    }
    c->tile_rows_all.insert(c->tile_rows_all.end(), P.tile_rows.begin(), P.tile_rows.end());
    c->tsten_all.insert(c->tsten_all.end(), P.tsten.begin(), P.tsten.end());
    c->ring_all.insert(c->ring_all.end(), P.ring.begin(), P.ring.end());
  }
  const int pL = c->L > 1 ? c->L - 1 : 0;
  gp_start[pL] = c->gp_all.size();
  tl_start[pL] = c->tiles_all.size();
  rg_start[pL] = c->ring_all.size();
  c->pair_gp.assign(c->pairs.size(), std::pair<size_t, size_t>(0, 0));
  for (size_t p = 0; p < c->pairs.size(); ++p) c->pair_gp[p] = {gp_start[p], gp_start[p + 1] - gp_start[p]};
  const int T = 1 << (c->L - 1);
  for (int t = 1; t <= T; ++t) {
    int lmin = c->L - 1;
    for (int l = 0; l < c->L; ++l)
      if (t % (1 << (c->L - 1 - l)) == 0) {
        lmin = l;
        break;
      }
    Tick tk;
    tk.lmin = lmin;
    tk.sc_off = c->sc_all.size();
    for (int l = lmin; l < c->L; ++l) {
      const auto &v = (l == lmin && l > 0) ? c->lev[l].items1 : c->lev[l].items2;
      c->sc_all.insert(c->sc_all.end(), v.begin(), v.end());
    }
    tk.sc_n = c->sc_all.size() - tk.sc_off;
    // plain bricks last: in one launch the costlier bricks (walls, interface layers,
    // boundaries) start first instead of forming the tail; the split modes take the
    // plain suffix
    auto mid = std::stable_partition(c->sc_all.begin() + tk.sc_off, c->sc_all.end(),
                                     [](const WorkItem &w) { return (w.flags & WI_PLAIN) == 0; });
    tk.sc_plain = (size_t)(c->sc_all.end() - mid);
    // XCD tables: workgroup q runs on XCD q mod 8, so position q takes a brick of group
    // q mod 8, the groups being slabs of each level along its slowest brick axis (z in
    // 3-D, y in 2-D) -- a brick's neighbours then share its XCD's L2 -- in item order
    // within a group (costlier bricks first); a group that runs out is helped by the
    // longest one
    auto table = [&](size_t r0, size_t n) {
      std::vector<std::vector<int32_t>> grp(8);
      for (size_t i = 0; i < n; ++i) {
        const WorkItem &w = c->sc_all[tk.sc_off + r0 + i];
        const Level &L = c->lev[w.level];
        const int ax = c->D == 3 ? 2 : 1;
        const int64_t bz = L.borg[(size_t)w.brick * 3 + ax] / bdim(c->D, ax);
        grp[(size_t)std::min<int64_t>(7, bz * 8 / std::max<int64_t>(1, L.gdim[ax]))].push_back((int32_t)i);
      }
      std::vector<size_t> head(8, 0);
      const size_t off = c->perm_all.size();
      for (size_t q = 0; q < n; ++q) {
        size_t g = q % 8;
        if (head[g] == grp[g].size()) {
          size_t best = 0;
          for (size_t k = 0; k < 8; ++k)
            if (grp[k].size() - head[k] > grp[best].size() - head[best]) best = k;
          g = best;
        }
        c->perm_all.push_back(grp[g][head[g]++]);
      }
      return off;
    };
    tk.pu_off = table(0, tk.sc_n);
    tk.ps_off = table(0, tk.sc_n - tk.sc_plain);
    tk.pp_off = table(tk.sc_n - tk.sc_plain, tk.sc_plain);
    const int p0 = std::min(lmin, pL);
    tk.gp_off = gp_start[p0];
    tk.gp_n = gp_start[pL] - tk.gp_off;
    tk.tile_off = tl_start[p0];
    tk.tile_n = tl_start[pL] - tk.tile_off;
    tk.ring_off = rg_start[p0];
    tk.ring_n = rg_start[pL] - tk.ring_off;
    c->ticks.push_back(tk);
  }
  // A gather launched in (level, brick, node) order has the lanes of a wavefront pull
  // from neighbouring nodes of one brick and runs ~1.4x faster than in first-use order;
  // that pays where the coupling branch is the longer one, while beside a longer
  // stream-collide the first-use order measured faster (channel: 1.3% per step).  So
  // the points of a pair are sorted if one of its ticks has the longer coupling branch.
  // Staging slots keep their first-use numbering (the rows one fine brick's stencils
  // read lie together), so the order changes no result.
  for (int p = 0; p + 1 < c->L; ++p) {
    bool sort = false;
    for (const Tick &tk : c->ticks) sort = sort || (std::min(tk.lmin, pL) <= p && coupling_longer(c, tk));
    if (!sort) continue;
    std::stable_sort(c->gp_all.begin() + (std::ptrdiff_t)gp_start[p], c->gp_all.begin() + (std::ptrdiff_t)gp_start[p + 1],
                     [](const GPoint &a, const GPoint &b) {
                       if (a.level != b.level) return a.level < b.level;
                       return a.brick != b.brick ? a.brick < b.brick : a.node < b.node;
                     });
  }
  c->red_items.clear();
  for (int l = 0; l < c->L; ++l)
    for (int32_t b = 0; b < c->lev[l].nb; ++b) {
      WorkItem w;
      w.brick = b;
      w.level = (uint8_t)l;
      w.thr = 0;
      w.drag = 0;
      w.flags = 0;
      c->red_items.push_back(w);
    }
}

size_t store_bytes(int st) { return st == ST_F64 ? 8 : (st == ST_F32 ? 4 : 2); }
size_t comp_bytes(int st) { return st == ST_F64 ? 8 : 4; }

void build_layout(elbm_ctx *c) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + std::max<size_t>(bytes, 1), 256);
    return o;
  };
  const size_t sb = store_bytes(c->storage);
  for (int l = 0; l < c->L; ++l) {
    Level &L = c->lev[l];
    const size_t nb = (size_t)L.nb;
    L.o_pop[0] = take(nb * c->Q * BN * sb);
    L.o_pop[1] = take(nb * c->Q * BN * sb);
    L.o_cls = take(nb * BN);
    L.o_mask = take(nb * BN * 4);
    L.o_w = take(nb * BN * 4);
    L.o_nbr = take(nb * 27 * 4);
    L.o_force = take(nb * c->D * BN * 4);
    L.o_gamma = take(nb * BN * 4);
    L.o_drag = take(nb * 3 * 8);
    L.o_borg = take(nb * 3 * 4);
  }
  c->o_levstatic = take(sizeof(LevelStatic) * MAXL);
  c->o_pairstatic = take(sizeof(PairStatic) * MAXL);
  c->o_sc = take(c->sc_all.size() * sizeof(ItemRec));
  c->o_perm = take(c->perm_all.size() * sizeof(int32_t));
  c->o_gp = take(c->gp_all.size() * sizeof(GPoint));
  c->o_fine = take(c->fine_all.size() * sizeof(CItem));
  c->o_ring = take(c->ring_all.size() * sizeof(CItem));
  c->o_tiles = take(c->tiles_all.size() * sizeof(CTile));
  c->o_trows = take(c->tile_rows_all.size() * sizeof(int32_t));
  c->o_sten = take(c->tsten_all.size() * sizeof(StencilEntry));
  c->o_stage = take((size_t)stage_row_width(c->D) * std::max(c->stage_cols, 1) * comp_bytes(c->storage));
  c->o_redit = take(c->red_items.size() * sizeof(WorkItem));
  c->o_part = take(c->red_items.size() * 5 * 8);
  c->o_res = take(8 * 8);
  c->tmp_bytes = 1 << 20;
  c->o_tmp = take(c->tmp_bytes);
  c->ws_need = off;
}

LevelStatic level_static(const elbm_ctx *c, int l) {
  const Level &L = c->lev[l];
  LevelStatic s;
  memset(&s, 0, sizeof(s));
  char *ws = c->ws;
  s.cls = (const uint8_t *)(ws + L.o_cls);
  s.mask = (const uint32_t *)(ws + L.o_mask);
  s.nbr = (const int32_t *)(ws + L.o_nbr);
  s.weight = (const float *)(ws + L.o_w);
  s.force = L.force_on ? (const float *)(ws + L.o_force) : nullptr;
  s.gamma = c->gamma_on ? (float *)(ws + L.o_gamma) : nullptr;
  s.drag = (double *)(ws + L.o_drag);
  s.beta = L.beta;
  const double sc = std::ldexp(1.0, -l);
  for (int a = 0; a < 3; ++a) s.F[a] = c->Fu[a] * sc;  // du_f = du_c / r (Sec. III.A)
  s.fscale = sc;
  int inlet = -1, outflow = -1;
  for (int f = 0; f < 6; ++f) {
    if (c->face_kind[f] == ELBM_FACE_INLET) inlet = f;
    if (c->face_kind[f] == ELBM_FACE_OUTFLOW) outflow = f;
  }
  if (inlet >= 0) heq_host(c->D, c->face_u[inlet], s.hin);
  if (outflow >= 0) s.oshift[outflow / 2] = (outflow & 1) ? 1 : -1;
  s.nbricks = L.nb;
  return s;
}

// The level and pair constants are read by every kernel: they are rewritten in order
// on the bound stream (after the work already enqueued there, which may still read the
// old values) and the call returns once the copy is done (the sources live on the host
// stack).
elbm_status upload_static(elbm_ctx *c) {
  LevelStatic ls[MAXL];
  memset(ls, 0, sizeof(ls));
  for (int l = 0; l < c->L; ++l) ls[l] = level_static(c, l);
  PairStatic ps[MAXL];
  memset(ps, 0, sizeof(ps));
  for (size_t p = 0; p < c->pairs.size(); ++p) {
    ps[p].fac_pc = c->pairs[p].fac_pc;
    ps[p].fac_cp = c->pairs[p].fac_cp;
    ps[p].parent = (int)p;
  }
  HIPCK(c, hipMemcpyAsync(c->ws + c->o_levstatic, ls, sizeof(ls), hipMemcpyHostToDevice, c->stream));
  HIPCK(c, hipMemcpyAsync(c->ws + c->o_pairstatic, ps, sizeof(ps), hipMemcpyHostToDevice, c->stream));
  HIPCK(c, hipStreamSynchronize(c->stream));
  return ELBM_OK;
}

// Executable graphs are destroyed only once nothing launched from them can still run:
// an earlier elbm_advance returns before its graph launches finish, and the runtime may
// run a graph's branches on streams of its own, so the whole device is waited for.
void invalidate_graphs(elbm_ctx *c) {
  bool any = false;
  for (int p = 0; p < 2; ++p) any = any || c->graph[p] || c->graphm[p];
  if (any) hipDeviceSynchronize();
  for (int p = 0; p < 2; ++p) {
    if (c->graph[p]) {
      hipGraphExecDestroy(c->graph[p]);
      c->graph[p] = nullptr;
    }
    if (c->graphm[p]) {
      hipGraphExecDestroy(c->graphm[p]);
      c->graphm[p] = nullptr;
    }
  }
  c->graph_valid = false;
}

// buffer index of level l at its k-th step (1-based) of a coarse step with level-0 parity p
int src_index(int l, int p, int k) { return ((l == 0 ? p : 0) ^ ((k - 1) & 1)); }

// one tick with explicit input/output buffers per level (flags: FL_DRAG, FL_GAMMA)
elbm_status enqueue_tick_io(elbm_ctx *c, int t, void *const src[MAXL], void *const dst[MAXL], hipStream_t main,
                            hipStream_t side, bool fork, int flags, void *stage = nullptr) {
  // staged rows of the tick's interpolation points: the context's buffer unless the
  // caller keeps them (the adjoint's recomputation)
  void *const stg = stage ? stage : (void *)(c->ws + c->o_stage);
  const Tick &tk = c->ticks[t - 1];
  const LevelStatic *lev = (const LevelStatic *)(c->ws + c->o_levstatic);
  const PairStatic *pairs = (const PairStatic *)(c->ws + c->o_pairstatic);
  const bool coupling = tk.tile_n + tk.ring_n > 0;
  hipStream_t cs = main;
  if (coupling && fork) {
    hipEvent_t ef = c->ev_fork[(t - 1) % 64];
    HIPCK(c, hipEventRecord(ef, main));
    HIPCK(c, hipStreamWaitEvent(side, ef, 0));
    cs = side;
  }
  // gather and coupling launches of the tick (on cs)
  auto couple = [&]() -> elbm_status {
    if (!coupling) return ELBM_OK;
    GatherArgs g;
    g.pts = (const GPoint *)(c->ws + c->o_gp) + tk.gp_off;
    g.n = (int)tk.gp_n;
    g.stride = stage_row_width(c->D);
    g.stage = stg;
    g.lev = lev;
    g.pairs = pairs;
    for (int l = 0; l < MAXL; ++l) {
      g.src[l] = src[l];
      g.nbr[l] = l < c->L ? (const int32_t *)(c->ws + c->lev[l].o_nbr) : nullptr;
    }
    LCK(c, launch_gather(c->D, c->storage, g, cs));
    CoupleArgs a;
    a.tiles = (const CTile *)(c->ws + c->o_tiles) + tk.tile_off;
    a.n_tiles = (int)tk.tile_n;
    a.lds_rows = c->lds_rows;
    a.lds_ents = c->lds_ents;
    a.tile_rows = (const int32_t *)(c->ws + c->o_trows);
    a.items = (const CItem *)(c->ws + c->o_fine);
    a.ring = (const CItem *)(c->ws + c->o_ring) + tk.ring_off;
    a.n_ring = (int)tk.ring_n;
    a.stride = stage_row_width(c->D);
    a.sten = (const StencilEntry *)(c->ws + c->o_sten);
    a.stage = stg;
    a.lev = lev;
    a.pairs = pairs;
    for (int l = 0; l < MAXL; ++l) {
      a.src[l] = src[l];
      a.dst[l] = dst[l];
    }
    a.flags = flags;
    a.lds_items = c->lds_items;
    LCK(c, launch_couple(c->D, c->storage, a, cs));
      return ELBM_OK;
  };
  SCArgs s;
  s.items = (const ItemRec *)(c->ws + c->o_sc) + tk.sc_off;
  s.n_items = (int)tk.sc_n;
  s.remap = c->xcd_remap;
  const int32_t *perm = (const int32_t *)(c->ws + c->o_perm);
  s.perm = c->xcd_remap == 1 ? perm + tk.pu_off : nullptr;
  s.flags = flags;
  s.pad = 0;
  s.lev = lev;
  for (int l = 0; l < MAXL; ++l) {
    s.src[l] = src[l];
    s.dst[l] = dst[l];
  }
  LaunchCfg cfg;
  cfg.threads = c->threads;
  cfg.occ = c->occ;
  cfg.pipe = 0;
  cfg.grid = c->wg_per_cu > 0 ? std::min<int>((int)tk.sc_n, c->wg_per_cu * c->cu_count) : (int)tk.sc_n;
  // split modes: plain bricks in a plain-only kernel (1: persistent pipelined, 2: one
  // node per thread within 128 VGPRs), the others (walls, interface layers,
  // inlet/outflow, drag) in the general kernel, one brick per workgroup
  SCArgs sp = s, sr = s;
  LaunchCfg cp = cfg, cr = cfg;
  const bool split = c->pipe && tk.sc_plain > 0;
  if (split) {
    sp.items = s.items + (tk.sc_n - tk.sc_plain);
    sp.n_items = (int)tk.sc_plain;
    sp.perm = c->xcd_remap == 1 ? perm + tk.pp_off : nullptr;
    sr.perm = c->xcd_remap == 1 ? perm + tk.ps_off : nullptr;
    cp.pipe = c->pipe;
    if (c->pipe == 1)
      cp.grid = std::min<int>((int)tk.sc_plain, (c->wg_per_cu > 0 ? c->wg_per_cu : 2) * c->cu_count);
    else
      cp.grid = c->wg_per_cu > 0 ? std::min<int>((int)tk.sc_plain, c->wg_per_cu * c->cu_count) : (int)tk.sc_plain;
    sr.n_items = (int)(tk.sc_n - tk.sc_plain);
    cr.grid = sr.n_items;
    cr.occ = 1;
    cr.threads = 256;
  }
  auto run = [&]() -> elbm_status {
    if (split && fork) {
      // in a graph the two launches are parallel branches (disjoint bricks, same inputs)
      hipEvent_t f2 = c->ev_fork2[(t - 1) % 64], j2 = c->ev_join2[(t - 1) % 64];
      HIPCK(c, hipEventRecord(f2, main));
      HIPCK(c, hipStreamWaitEvent(c->side2, f2, 0));
      LCK(c, launch_stream_collide(c->D, c->storage, sr, cr, c->side2));
      LCK(c, launch_stream_collide(c->D, c->storage, sp, cp, main));
      HIPCK(c, hipEventRecord(j2, c->side2));
      HIPCK(c, hipStreamWaitEvent(main, j2, 0));
    } else if (split) {
      LCK(c, launch_stream_collide(c->D, c->storage, sr, cr, main));
      LCK(c, launch_stream_collide(c->D, c->storage, sp, cp, main));
    } else {
      LCK(c, launch_stream_collide(c->D, c->storage, s, cfg, main));
    }
    return ELBM_OK;
  };
  // In a graph the graph executor keeps the first-captured dependent of a node on that
  // node's queue; a dependency across queues costs 5-10 us.  So the longer of the two
  // branches of a coupling tick is captured first and stays on the queue of the
  // previous tick's stream-collide.
  const bool sc_first = fork && coupling && !coupling_longer(c, tk);
  if (!sc_first) {
    elbm_status st = couple();
    if (st) return st;
  }
  if (c->timing) {
    hipEvent_t e0, e1;
    HIPCK(c, hipEventCreate(&e0));
    HIPCK(c, hipEventCreate(&e1));
    c->tev.push_back(e0);
    c->tev.push_back(e1);
    if (!split && s.n_items > 0) {
      // one launch: its dispatch packet stamps the events with the kernel's own start
      // and end, as a kernel tracer reports it (a tick without items launches nothing,
      // and its events are recorded below, back to back)
      cfg.ev0 = e0;
      cfg.ev1 = e1;
      elbm_status st = run();
      cfg.ev0 = cfg.ev1 = nullptr;
      if (st) return st;
    } else {
      HIPCK(c, hipEventRecord(e0, main));
      elbm_status st = run();
      if (st) return st;
      HIPCK(c, hipEventRecord(e1, main));
    }
  } else {
    elbm_status st = run();
    if (st) return st;
  }
  if (sc_first) {
    elbm_status st = couple();
    if (st) return st;
  }
  if (coupling && fork) {
    hipEvent_t ej = c->ev_join[(t - 1) % 64];
    HIPCK(c, hipEventRecord(ej, side));
    HIPCK(c, hipStreamWaitEvent(main, ej, 0));
  }
  return ELBM_OK;
}

elbm_status enqueue_tick(elbm_ctx *c, int t, int p, hipStream_t main, hipStream_t side, bool fork) {
  const Tick &tk = c->ticks[t - 1];
  void *src[MAXL] = {}, *dst[MAXL] = {};
  for (int l = tk.lmin; l < c->L; ++l) {
    const int k = t >> (c->L - 1 - l);
    const int si = src_index(l, p, k);
    src[l] = c->ws + c->lev[l].o_pop[si];
    dst[l] = c->ws + c->lev[l].o_pop[si ^ 1];
  }
  return enqueue_tick_io(c, t, src, dst, main, side, fork, FL_DRAG | FL_GAMMA);
}

elbm_status enqueue_coarse_step(elbm_ctx *c, int p, hipStream_t main, hipStream_t side, bool fork) {
  const int T = 1 << (c->L - 1);
  for (int t = 1; t <= T; ++t) {
    elbm_status s = enqueue_tick(c, t, p, main, side, fork);
    if (s) return s;
  }
  return ELBM_OK;
}

// capture `steps` consecutive coarse steps starting at level-0 parity p
elbm_status capture_steps(elbm_ctx *c, int p, int steps, hipGraphExec_t *out) {
  HIPCK(c, hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
  elbm_status s = ELBM_OK;
  for (int k = 0; k < steps && !s; ++k) s = enqueue_coarse_step(c, p ^ (k & 1), c->cap, c->side, true);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(c->cap, &g);
  if (s) {
    if (g) hipGraphDestroy(g);
    return s;
  }
  if (e != hipSuccess) FAIL(c, ELBM_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
  e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  if (e != hipSuccess) FAIL(c, ELBM_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
  return ELBM_OK;
}

elbm_status build_graphs(elbm_ctx *c) {
  invalidate_graphs(c);
  for (int p = 0; p < 2; ++p) {
    elbm_status s = capture_steps(c, p, 1, &c->graph[p]);
    if (!s && c->use_graph > 1) s = capture_steps(c, p, c->use_graph, &c->graphm[p]);
    if (s) return s;
  }
  c->graph_valid = true;
  return ELBM_OK;
}

elbm_status check_level(const elbm_ctx *c, int level) {
  if (!c->finalized) return ELBM_ESTATE;
  if (level < 0 || level >= c->L) return ELBM_EINVAL;
  return ELBM_OK;
}


// ---------------------------------------------------------------- discrete adjoint (host)
// Reverse sweep of the coarse step: segments of K coarse steps are recomputed from
// checkpoints into a tape of per-substep states (one slot per level substep), then
// the ticks are reversed one by one (kernels in adjoint.hip).

void adj_build_tables(elbm_ctx *c) {
  auto &A = c->adj;
  A.items.clear();
  A.tick.clear();
  const int T = 1 << (c->L - 1);
  for (int t = 1; t <= T; ++t) {
    const int lmin = c->ticks[t - 1].lmin;
    const size_t off = A.items.size();
    for (int l = lmin; l < c->L; ++l)
      for (int32_t b = 0; b < c->lev[l].nb; ++b) {
        WorkItem w;
        w.brick = b;
        w.level = (uint8_t)l;
        w.thr = (uint8_t)((l == lmin && l > 0) ? 1 : 2);
        w.drag = 0;
        w.flags = 0;
        A.items.push_back(w);
      }
    A.tick.push_back({off, A.items.size() - off});
  }
  A.bitems.clear();
  A.btick.clear();
  for (int t = 1; t <= T; ++t) {
    const int tp = t > 1 ? t - 1 : T;
    const int lt = c->ticks[t - 1].lmin, lp = c->ticks[tp - 1].lmin;
    const size_t off = A.bitems.size();
    for (int l = std::min(lt, lp); l < c->L; ++l)
      for (int32_t b = 0; b < c->lev[l].nb; ++b) {
        WorkItem w;
        w.brick = b;
        w.level = (uint8_t)l;
        w.thr = (uint8_t)(l < lp ? 0 : ((l == lp && l > 0) ? 1 : 2));
        w.drag = 0;
        w.flags = 0;
        A.bitems.push_back(w);
      }
    A.btick.push_back({off, A.bitems.size() - off});
  }
  // transposed interpolation stencils: per staged row, the fine items reading it
  const int ncols = std::max(c->stage_cols, 1);
  std::vector<std::vector<StencilEntry>> by((size_t)ncols);
  for (const CTile &t : c->tiles_all)
    for (int32_t k = 0; k < t.nitem; ++k) {
      const int32_t item = t.item0 + k;
      const CItem &it = c->fine_all[(size_t)item];
      for (int32_t e = it.a; e < it.a + it.b; ++e) {
        const StencilEntry &se = c->tsten_all[(size_t)e];
        StencilEntry o;
        o.slot = item;
        o.w = se.w;
        by[(size_t)c->tile_rows_all[(size_t)(t.pt0 + se.slot)]].push_back(o);
      }
    }
  A.tofs.assign((size_t)ncols + 1, 0);
  A.tsten.clear();
  for (int k = 0; k < ncols; ++k) {
    A.tofs[(size_t)k] = (int32_t)A.tsten.size();
    A.tsten.insert(A.tsten.end(), by[(size_t)k].begin(), by[(size_t)k].end());
  }
  A.tofs[(size_t)ncols] = (int32_t)A.tsten.size();
  // populations that outflow nodes copy from their upstream neighbour
  int outflow = -1;
  for (int f = 0; f < 6; ++f)
    if (c->face_kind[f] == ELBM_FACE_OUTFLOW) outflow = f;
  for (int l = 0; l < c->L; ++l) {
    A.has_amask[l] = false;
    A.amask[l].clear();
  }
  if (outflow < 0) return;
  int64_t osh[3] = {0, 0, 0};
  osh[outflow / 2] = (outflow & 1) ? 1 : -1;
  for (int l = 0; l < c->L; ++l) {
    const Level &L = c->lev[l];
    A.amask[l].assign((size_t)L.nb * BN, 0u);
    for (int32_t b = 0; b < L.nb; ++b)
      for (int n = 0; n < BN; ++n) {
        const size_t k = (size_t)b * BN + n;
        if (!(L.cls[k] & CLS_FLUID)) continue;
        const int64_t loc[3] = {n % bdim(c->D, 0), (n / bdim(c->D, 0)) % bdim(c->D, 1),
                                n / (bdim(c->D, 0) * bdim(c->D, 1))};
        for (int i = 0; i < c->Q; ++i) {
          int64_t y[3];
          for (int a = 0; a < 3; ++a) y[a] = L.blo[a] + L.borg[3 * b + a] + loc[a] + vel(c->D, i, a) + osh[a];
          NodeRef r = locate(c, l, y);
          if (r.brick < 0) continue;
          const size_t m = (size_t)r.brick * BN + r.node;
          if ((L.cls[m] & CLS_OUTFLOW) && ((L.mask[m] >> i) & 1u)) A.amask[l][k] |= 1u << i;
        }
        if (A.amask[l][k]) A.has_amask[l] = true;
      }
  }
}

size_t level_state_bytes(const elbm_ctx *c, int l) {
  return (size_t)c->lev[l].nb * c->Q * BN * store_bytes(c->storage);
}

void adj_layout(elbm_ctx *c, int nmax, int K) {
  auto &A = c->adj;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + std::max<size_t>(bytes, 1), 256);
    return o;
  };
  const size_t tb = comp_bytes(c->storage);
  size_t state = 0;
  for (int l = 0; l < c->L; ++l) {
    for (int q = 0; q < 2; ++q) A.o_tape[q][l] = take(level_state_bytes(c, l) * ((size_t)K * ((size_t)1 << l) + 1));
    state += level_state_bytes(c, l);
  }
  const size_t S = (size_t)((nmax + K - 1) / K);
  A.o_ckpt = take(S * state);
  for (int l = 0; l < c->L; ++l) {
    const size_t nb = (size_t)c->lev[l].nb;
    A.o_lam[l][0] = take(nb * c->Q * BN * tb);
    A.o_lam[l][1] = take(nb * c->Q * BN * tb);
    A.o_lg[l][0] = take((nb + 1) * c->Q * BN * tb);
    A.o_lg[l][1] = take((nb + 1) * c->Q * BN * tb);
    A.o_lF[l] = take(nb * c->D * BN * tb);
    A.o_amask[l] = take(A.has_amask[l] ? nb * BN * 4 : 0);
  }
  A.o_alev = take(sizeof(AdjLevel) * MAXL);
  A.o_astage = take(c->fine_all.size() * stage_row_width(c->D) * tb);
  const int T = 1 << (c->L - 1);
  A.ctick.assign((size_t)T, -1);
  A.nct = 0;
  for (int t = 1; t <= T; ++t)
    if (c->ticks[(size_t)t - 1].tile_n + c->ticks[(size_t)t - 1].ring_n > 0) A.ctick[(size_t)t - 1] = A.nct++;
  A.stage_bytes = align_up((size_t)stage_row_width(c->D) * std::max(c->stage_cols, 1) * tb, 256);
  for (int q = 0; q < 2; ++q) A.o_stape[q] = take((size_t)K * A.nct * A.stage_bytes);
  A.o_tofs = take(A.tofs.size() * 4);
  A.o_tsten = take(A.tsten.size() * sizeof(StencilEntry));
  A.o_items = take(A.items.size() * sizeof(WorkItem));
  A.o_bitems = take(A.bitems.size() * sizeof(WorkItem));
  A.o_part = take(c->red_items.size() * 5 * 8);
  A.o_res = take(64);
  A.need = off;
}

// staged rows of coupling tick t of coarse step k (1-based) of a segment, in tape set q
char *adj_stage(elbm_ctx *c, int q, int k, int t) {
  auto &A = c->adj;
  return A.ws + A.o_stape[q] + ((size_t)(k - 1) * A.nct + (size_t)A.ctick[(size_t)t - 1]) * A.stage_bytes;
}

char *adj_tape(elbm_ctx *c, int q, int l, size_t slot) {
  return c->adj.ws + c->adj.o_tape[q][l] + slot * level_state_bytes(c, l);
}

char *adj_ckpt(elbm_ctx *c, int s, int l) {
  size_t state = 0, before = 0;
  for (int q = 0; q < c->L; ++q) {
    if (q < l) before += level_state_bytes(c, q);
    state += level_state_bytes(c, q);
  }
  return c->adj.ws + c->adj.o_ckpt + (size_t)s * state + before;
}

char *cur_state(elbm_ctx *c, int l) { return c->ws + c->lev[l].o_pop[l == 0 ? c->parity : 0]; }

// Reverse sweep, tick by tick in reverse order.  Each level keeps two lam buffers (cur:
// the adjoint of its current state) and two lg buffers (lgc: its latest collision
// adjoint).  Reversing a tick t: (first tick of the run only) the collision adjoint;
// the coupling and interpolation-point adjoints of t; then one fused launch with the
// streaming transpose of t and the collision adjoint of the tick before it
// (k_adj_tc), or the transpose alone after the first tick of the run.

// tape slot of level l at tick t of coarse step k (1-based) of a segment
size_t tape_slot(const elbm_ctx *c, int l, int k, int t) {
  return ((size_t)(k - 1) << l) + (size_t)((t >> (c->L - 1 - l)) - 1);
}

void adj_fill_common(elbm_ctx *c, AdjArgs &a) {
  auto &A = c->adj;
  a.drag_level = A.objective == ELBM_OBJ_DRAG ? A.body_level : -1;
  if (A.objective == ELBM_OBJ_DRAG) {
    const double nsub = (double)A.n * (double)((int64_t)1 << A.body_level);
    for (int q = 0; q < 3; ++q) a.drag_seed[q] = A.dir[q] / nsub;
  }
  a.lev = (const LevelStatic *)(c->ws + c->o_levstatic);
  a.alev = (const AdjLevel *)(A.ws + A.o_alev);
}

// collision adjoint of tick t of coarse step k (the first reversed tick of the run)
elbm_status adj_collide_first(elbm_ctx *c, int k, int t) {
  auto &A = c->adj;
  AdjArgs a;
  memset(&a, 0, sizeof(a));
  adj_fill_common(c, a);
  a.items = (const WorkItem *)(A.ws + A.o_items) + A.tick[(size_t)t - 1].first;
  a.n_items = (int)A.tick[(size_t)t - 1].second;
  for (int l = 0; l < c->L; ++l) {
    a.lg[l] = A.ws + A.o_lg[l][A.lgc[l]];
    a.lF[l] = A.ws + A.o_lF[l];
  }
  for (int l = c->ticks[t - 1].lmin; l < c->L; ++l) {
    a.src[l] = adj_tape(c, A.rset, l, tape_slot(c, l, k, t));
    a.lam[l] = A.ws + A.o_lam[l][A.cur[l]];
  }
  LCK(c, launch_adj_collide(c->D, c->storage, a, c->stream));
  return ELBM_OK;
}

// coupling and interpolation-point adjoints of tick t of coarse step k
elbm_status adj_couple_part(elbm_ctx *c, int k, int t) {
  auto &A = c->adj;
  const Tick &tk = c->ticks[t - 1];
  if (tk.tile_n + tk.ring_n == 0) return ELBM_OK;
  const int L = c->L;
  const LevelStatic *lev = (const LevelStatic *)(c->ws + c->o_levstatic);
  const PairStatic *pairs = (const PairStatic *)(c->ws + c->o_pairstatic);
  void *src[MAXL] = {};
  for (int l = tk.lmin; l < L; ++l) src[l] = adj_tape(c, A.rset, l, tape_slot(c, l, k, t));
  // the staged rows of this tick were kept by the recomputation
  AdjCoupleArgs ca;
  memset(&ca, 0, sizeof(ca));
  ca.c.tiles = (const CTile *)(c->ws + c->o_tiles) + tk.tile_off;
  ca.c.n_tiles = (int)tk.tile_n;
  ca.c.lds_rows = c->lds_rows;
  ca.c.lds_ents = c->lds_ents;
  ca.c.tile_rows = (const int32_t *)(c->ws + c->o_trows);
  ca.c.items = (const CItem *)(c->ws + c->o_fine);
  ca.c.ring = (const CItem *)(c->ws + c->o_ring) + tk.ring_off;
  ca.c.n_ring = (int)tk.ring_n;
  ca.c.stride = stage_row_width(c->D);
  ca.c.sten = (const StencilEntry *)(c->ws + c->o_sten);
  ca.c.stage = adj_stage(c, A.rset, k, t);
  ca.c.lev = lev;
  ca.c.pairs = pairs;
  for (int l = 0; l < MAXL; ++l) {
    ca.c.src[l] = src[l];
    if (l < L) {
      ca.lam[l] = A.ws + A.o_lam[l][A.cur[l]];
      ca.lg[l] = A.ws + A.o_lg[l][A.lgc[l]];
      ca.lF[l] = A.ws + A.o_lF[l];
    }
  }
  ca.astage = A.ws + A.o_astage;
  LCK(c, launch_adj_couple(c->D, c->storage, ca, c->stream));
  // pairs one after the other: a level's points of two pairs may coincide
  for (int p = tk.lmin; p + 1 < L; ++p) {
    AdjPointArgs pa;
    memset(&pa, 0, sizeof(pa));
    pa.pts = (const GPoint *)(c->ws + c->o_gp) + c->pair_gp[(size_t)p].first;
    pa.n = (int)c->pair_gp[(size_t)p].second;
    pa.tofs = (const int32_t *)(A.ws + A.o_tofs);
    pa.tsten = (const StencilEntry *)(A.ws + A.o_tsten);
    pa.astage = A.ws + A.o_astage;
    pa.lev = lev;
    pa.pairs = pairs;
    for (int l = 0; l < MAXL; ++l) {
      pa.src[l] = src[l];
      if (l < L) pa.lg[l] = A.ws + A.o_lg[l][A.lgc[l]];
    }
    LCK(c, launch_adj_points(c->D, c->storage, pa, c->stream));
  }
  return ELBM_OK;
}

// streaming transpose of tick t fused with the collision adjoint of the tick before it
// (t - 1 of the same coarse step, or T of coarse step kp = k - 1), read from tape set q
elbm_status adj_boundary(elbm_ctx *c, int t, int kp, int q) {
  auto &A = c->adj;
  const int T = 1 << (c->L - 1);
  const int tp = t > 1 ? t - 1 : T;
  const int lt = c->ticks[t - 1].lmin, lp = c->ticks[tp - 1].lmin;
  AdjTCArgs a;
  memset(&a, 0, sizeof(a));
  a.items = (const WorkItem *)(A.ws + A.o_bitems) + A.btick[(size_t)t - 1].first;
  a.n_items = (int)A.btick[(size_t)t - 1].second;
  a.drag_level = A.objective == ELBM_OBJ_DRAG ? A.body_level : -1;
  if (A.objective == ELBM_OBJ_DRAG) {
    const double nsub = (double)A.n * (double)((int64_t)1 << A.body_level);
    for (int d = 0; d < 3; ++d) a.drag_seed[d] = A.dir[d] / nsub;
  }
  a.lev = (const LevelStatic *)(c->ws + c->o_levstatic);
  a.alev = (const AdjLevel *)(A.ws + A.o_alev);
  for (int l = std::min(lt, lp); l < c->L; ++l) {
    const bool tr = l >= lt, co = l >= lp;
    if (tr) a.tpose_mask |= 1u << l;
    if (co) a.coll_mask |= 1u << l;
    a.lgsrc[l] = A.ws + A.o_lg[l][A.lgc[l]];
    a.lam[l] = A.ws + A.o_lam[l][tr ? A.cur[l] ^ 1 : A.cur[l]];
    a.lgdst[l] = A.ws + A.o_lg[l][A.lgc[l] ^ 1];
    a.lF[l] = A.ws + A.o_lF[l];
    if (co) a.src[l] = adj_tape(c, q, l, tape_slot(c, l, kp, tp));
  }
  LCK(c, launch_adj_tc(c->D, c->storage, a, c->stream));
  for (int l = std::min(lt, lp); l < c->L; ++l) {
    if (l >= lt) A.cur[l] ^= 1;
    if (l >= lp) A.lgc[l] ^= 1;
  }
  return ELBM_OK;
}

// streaming transpose alone (the first tick of the run, reversed last)
elbm_status adj_transpose_last(elbm_ctx *c, int t) {
  auto &A = c->adj;
  AdjArgs a;
  memset(&a, 0, sizeof(a));
  adj_fill_common(c, a);
  a.items = (const WorkItem *)(A.ws + A.o_items) + A.tick[(size_t)t - 1].first;
  a.n_items = (int)A.tick[(size_t)t - 1].second;
  for (int l = c->ticks[t - 1].lmin; l < c->L; ++l) {
    a.lg[l] = A.ws + A.o_lg[l][A.lgc[l]];
    a.lam[l] = A.ws + A.o_lam[l][A.cur[l] ^ 1];
  }
  LCK(c, launch_adj_transpose(c->D, c->storage, a, c->stream));
  for (int l = c->ticks[t - 1].lmin; l < c->L; ++l) A.cur[l] ^= 1;
  return ELBM_OK;
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

const char *elbm_status_string(elbm_status s) {
  switch (s) {
    case ELBM_OK: return "ok";
    case ELBM_EINVAL: return "invalid argument or geometry";
    case ELBM_ESTATE: return "call out of order";
    case ELBM_ESMALL: return "workspace too small";
    case ELBM_EDEVICE: return "HIP runtime error";
    case ELBM_EUNSTABLE: return "unstable state";
    case ELBM_ENOMEM: return "out of host memory";
  }
  return "unknown status";
}

const char *elbm_last_error(const elbm_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

elbm_status elbm_create(const elbm_desc *d, elbm_ctx **out) {
  if (!d || !out) return ELBM_EINVAL;
  *out = nullptr;
  if (d->dim != 2 && d->dim != 3) return ELBM_EINVAL;
  if (d->storage < ST_F64 || d->storage > ST_BF16S) return ELBM_EINVAL;
  if (d->n_levels < 1 || d->n_levels > MAXL) return ELBM_EINVAL;
  if (!(d->nu0 > 0)) return ELBM_EINVAL;
  elbm_ctx *c = new (std::nothrow) elbm_ctx();
  if (!c) return ELBM_ENOMEM;
  c->D = d->dim;
  c->Q = d->dim == 2 ? 9 : 27;
  c->L = d->n_levels;
  c->storage = d->storage;
  c->nu0 = d->nu0;
  for (int a = 0; a < 3; ++a) {
    c->N[a] = a < c->D ? d->extent[a] : 1;
    c->periodic[a] = a < c->D ? (d->periodic[a] != 0) : 0;
    if (a < c->D && c->N[a] < 2) {
      delete c;
      return ELBM_EINVAL;
    }
  }
  for (int f = 0; f < 6; ++f) c->face_kind[f] = (f / 2 < c->D && !c->periodic[f / 2]) ? ELBM_FACE_WALL : 0;
  *out = c;
  return ELBM_OK;
}

elbm_status elbm_destroy(elbm_ctx *c) {
  if (!c) return ELBM_EINVAL;
  // work enqueued by this context (graph launches included) ends before its graphs,
  // events and streams are released
  if (c->bound) hipStreamSynchronize(c->stream);
  if (c->side) hipStreamSynchronize(c->side);
  if (c->side2) hipStreamSynchronize(c->side2);
  invalidate_graphs(c);
  for (hipEvent_t e : c->tev) hipEventDestroy(e);
  for (int i = 0; i < c->n_events; ++i) {
    hipEventDestroy(c->ev_fork[i]);
    hipEventDestroy(c->ev_join[i]);
    hipEventDestroy(c->ev_fork2[i]);
    hipEventDestroy(c->ev_join2[i]);
  }
  if (c->side) hipStreamDestroy(c->side);
  if (c->cap) hipStreamDestroy(c->cap);
  if (c->side2) hipStreamDestroy(c->side2);
  delete c;
  return ELBM_OK;
}

elbm_status elbm_set_face(elbm_ctx *c, int face, int kind, const double u[3]) {
  if (!c) return ELBM_EINVAL;
  if (c->finalized) FAIL(c, ELBM_ESTATE, "set_face after finalize");
  if (face < 0 || face >= 6 || face / 2 >= c->D) FAIL(c, ELBM_EINVAL, "bad face %d", face);
  if (c->periodic[face / 2]) FAIL(c, ELBM_EINVAL, "face %d is on a periodic axis", face);
  if (kind < ELBM_FACE_WALL || kind > ELBM_FACE_OUTFLOW) FAIL(c, ELBM_EINVAL, "bad face kind %d", kind);
  for (int f = 0; f < 6; ++f)
    if (f != face && kind != ELBM_FACE_WALL && c->face_kind[f] == kind)
      FAIL(c, ELBM_EINVAL, "only one inlet and one outflow face are supported");
  c->face_kind[face] = kind;
  for (int a = 0; a < 3; ++a) c->face_u[face][a] = u ? u[a] : 0.0;
  return ELBM_OK;
}

elbm_status elbm_add_block(elbm_ctx *c, int level, const int64_t lo[3], const int64_t hi[3]) {
  if (!c || !lo || !hi) return ELBM_EINVAL;
  if (c->finalized) FAIL(c, ELBM_ESTATE, "add_block after finalize");
  if (level < 1 || level >= c->L) FAIL(c, ELBM_EINVAL, "blocks are added to levels 1..%d", c->L - 1);
  Box b;
  for (int a = 0; a < 3; ++a) {
    b.lo[a] = a < c->D ? lo[a] : 0;
    b.hi[a] = a < c->D ? hi[a] : 0;
  }
  for (int a = 0; a < c->D; ++a) {
    if (b.hi[a] < b.lo[a]) FAIL(c, ELBM_EINVAL, "empty block on axis %d", a);
    if (c->periodic[a]) {
      const int64_t P = period(c, level, a);
      if (b.lo[a] < 0 || b.lo[a] >= P || b.hi[a] - b.lo[a] > P - 1)
        FAIL(c, ELBM_EINVAL, "block outside the periodic range on axis %d", a);
      if (b.hi[a] - b.lo[a] == P - 1) continue;
    } else if (b.lo[a] < 0 || b.hi[a] > extent(c, level, a) - 1) {
      FAIL(c, ELBM_EINVAL, "block outside the domain on axis %d", a);
    }
    if ((b.lo[a] & 1) || (b.hi[a] & 1))
      FAIL(c, ELBM_EINVAL, "block faces must lie on parent nodes (even coordinates), axis %d", a);
    if (b.hi[a] - b.lo[a] < 8) FAIL(c, ELBM_EINVAL, "block narrower than 4 parent spacings on axis %d", a);
  }
  c->lev[level].boxes.push_back(b);
  return ELBM_OK;
}

elbm_status elbm_set_solid(elbm_ctx *c, int level, const int64_t lo[3], const int64_t n[3], const uint8_t *mask) {
  if (!c || !lo || !n || !mask) return ELBM_EINVAL;
  if (c->finalized) FAIL(c, ELBM_ESTATE, "set_solid after finalize");
  if (level < 0 || level >= c->L) FAIL(c, ELBM_EINVAL, "bad level %d", level);
  SolidSpec s;
  size_t tot = 1;
  for (int a = 0; a < 3; ++a) {
    s.lo[a] = a < c->D ? lo[a] : 0;
    s.n[a] = a < c->D ? n[a] : 1;
    if (s.n[a] < 1) FAIL(c, ELBM_EINVAL, "bad solid extent");
    tot *= (size_t)s.n[a];
  }
  s.mask.assign(mask, mask + tot);
  c->lev[level].solids.push_back(std::move(s));
  return ELBM_OK;
}

elbm_status elbm_set_force_uniform(elbm_ctx *c, const double F[3]) {
  if (!c || !F) return ELBM_EINVAL;
  for (int a = 0; a < 3; ++a) c->Fu[a] = a < c->D ? F[a] : 0.0;
  if (c->bound) {
    elbm_status s = upload_static(c);
    if (s) return s;
    invalidate_graphs(c);
  }
  return ELBM_OK;
}

elbm_status elbm_finalize(elbm_ctx *c, size_t *ws_bytes) {
  if (!c) return ELBM_EINVAL;
  if (c->finalized) FAIL(c, ELBM_ESTATE, "finalize twice");
  for (int l = 1; l < c->L; ++l)
    if (c->lev[l].boxes.empty()) FAIL(c, ELBM_EINVAL, "level %d has no blocks", l);
  try {
    for (int l = 0; l < c->L; ++l) {
      elbm_status s = build_level_geometry(c, l);
      if (s) return s;
    }
    for (int l = 0; l < c->L; ++l) {
      elbm_status s = build_level_links(c, l);
      if (s) return s;
    }
    // a parent ring node must not lie on the parent's own interface layers
    for (int l = 0; l < c->L; ++l) {
      const Level &L = c->lev[l];
      for (size_t k = 0; k < L.exists.size(); ++k)
        if (L.exists[k] && L.ring[k] && L.pd[k] < 2)
          FAIL(c, ELBM_EINVAL, "level %d: a ring node lies on the level's own interface (nesting margin)", l);
    }
    elbm_status s = build_pairs(c);
    if (s) return s;
    build_schedule(c);
    for (int l = 0; l < c->L; ++l)
      if ((double)c->lev[l].nb * c->Q * BN * store_bytes(c->storage) >= 4294967296.0)
        FAIL(c, ELBM_EINVAL, "level %d population buffer exceeds 4 GiB (32-bit offsets)", l);
    build_layout(c);
  } catch (const std::bad_alloc &) {
    FAIL(c, ELBM_ENOMEM, "host allocation failed in finalize");
  }
  c->finalized = true;
  if (ws_bytes) *ws_bytes = c->ws_need;
  return ELBM_OK;
}

elbm_status elbm_level_box(const elbm_ctx *c, int level, int64_t lo[3], int64_t n[3]) {
  if (!c || !lo || !n) return ELBM_EINVAL;
  elbm_status s = check_level(c, level);
  if (s) return s;
  for (int a = 0; a < 3; ++a) {
    lo[a] = c->lev[level].blo[a];
    n[a] = c->lev[level].bn[a];
  }
  return ELBM_OK;
}

elbm_status elbm_level_info(const elbm_ctx *c, int level, int64_t *n_nodes, int64_t *n_fluid, double *beta,
                            int64_t *n_bricks) {
  if (!c) return ELBM_EINVAL;
  elbm_status s = check_level(c, level);
  if (s) return s;
  const Level &L = c->lev[level];
  if (n_nodes) *n_nodes = L.n_nodes;
  if (n_fluid) *n_fluid = L.n_fluid;
  if (beta) *beta = L.beta;
  if (n_bricks) *n_bricks = L.nb;
  return ELBM_OK;
}

static void dense_index(const elbm_ctx *c, int level, int32_t b, int n, int64_t &k, bool &in) {
  const Level &L = c->lev[level];
  int64_t loc[3] = {n % bdim(c->D, 0), (n / bdim(c->D, 0)) % bdim(c->D, 1), n / (bdim(c->D, 0) * bdim(c->D, 1))};
  int64_t X = L.borg[3 * b] + loc[0], Y = L.borg[3 * b + 1] + loc[1], Z = L.borg[3 * b + 2] + loc[2];
  in = X < L.bn[0] && Y < L.bn[1] && Z < L.bn[2];
  k = X + L.bn[0] * (Y + L.bn[1] * Z);
}

elbm_status elbm_node_class(const elbm_ctx *c, int level, int32_t *out) {
  if (!c || !out) return ELBM_EINVAL;
  elbm_status s = check_level(c, level);
  if (s) return s;
  const Level &L = c->lev[level];
  const int64_t tot = L.bn[0] * L.bn[1] * L.bn[2];
  for (int64_t k = 0; k < tot; ++k) out[k] = -1;
  for (int32_t b = 0; b < L.nb; ++b)
    for (int n = 0; n < BN; ++n) {
      const size_t q = (size_t)b * BN + n;
      if (!L.exists[q]) continue;
      int64_t k;
      bool in;
      dense_index(c, level, b, n, k, in);
      if (!in) continue;
      out[k] = (int32_t)(L.solid[q] | (L.ring[q] << 1) | (std::min<int>(L.pd[q], 3) << 2));
    }
  return ELBM_OK;
}

elbm_status elbm_weights(const elbm_ctx *c, int level, double *out) {
  if (!c || !out) return ELBM_EINVAL;
  elbm_status s = check_level(c, level);
  if (s) return s;
  const Level &L = c->lev[level];
  const int64_t tot = L.bn[0] * L.bn[1] * L.bn[2];
  for (int64_t k = 0; k < tot; ++k) out[k] = 0.0;
  for (int32_t b = 0; b < L.nb; ++b)
    for (int n = 0; n < BN; ++n) {
      const size_t q = (size_t)b * BN + n;
      if (!L.exists[q]) continue;
      int64_t k;
      bool in;
      dense_index(c, level, b, n, k, in);
      if (in) out[k] = L.weight[q];
    }
  return ELBM_OK;
}

elbm_status elbm_bind(elbm_ctx *c, void *ws, size_t bytes, void *stream) {
  if (!c || !ws) return ELBM_EINVAL;
  if (!c->finalized) FAIL(c, ELBM_ESTATE, "bind before finalize");
  if (bytes < c->ws_need) FAIL(c, ELBM_ESMALL, "workspace %zu bytes < %zu required", bytes, c->ws_need);
  if ((uintptr_t)ws & 255) FAIL(c, ELBM_EINVAL, "workspace must be 256-byte aligned");
  invalidate_graphs(c);
  c->ws = (char *)ws;
  c->stream = (hipStream_t)stream;
  int dev = 0;
  HIPCK(c, hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIPCK(c, hipGetDeviceProperties(&prop, dev));
  c->cu_count = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  HIPCK(c, static_staging_address(dev, &c->static_staging));
  if (!c->side) HIPCK(c, hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
  if (!c->cap) HIPCK(c, hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
  if (!c->side2) HIPCK(c, hipStreamCreateWithFlags(&c->side2, hipStreamNonBlocking));
  if (!c->n_events) {
    for (int i = 0; i < 64; ++i) {
      HIPCK(c, hipEventCreateWithFlags(&c->ev_fork[i], hipEventDisableTiming));
      HIPCK(c, hipEventCreateWithFlags(&c->ev_join[i], hipEventDisableTiming));
      HIPCK(c, hipEventCreateWithFlags(&c->ev_fork2[i], hipEventDisableTiming));
      HIPCK(c, hipEventCreateWithFlags(&c->ev_join2[i], hipEventDisableTiming));
    }
    c->n_events = 64;
  }
  for (int l = 0; l < c->L; ++l) {
    Level &L = c->lev[l];
    HIPCK(c, hipMemcpy(c->ws + L.o_cls, L.cls.data(), L.cls.size(), hipMemcpyHostToDevice));
    HIPCK(c, hipMemcpy(c->ws + L.o_mask, L.mask.data(), L.mask.size() * 4, hipMemcpyHostToDevice));
    HIPCK(c, hipMemcpy(c->ws + L.o_w, L.weight.data(), L.weight.size() * 4, hipMemcpyHostToDevice));
    HIPCK(c, hipMemcpy(c->ws + L.o_nbr, L.nbr.data(), L.nbr.size() * 4, hipMemcpyHostToDevice));
    HIPCK(c, hipMemcpy(c->ws + L.o_borg, L.borg.data(), L.borg.size() * 4, hipMemcpyHostToDevice));
    HIPCK(c, hipMemset(c->ws + L.o_drag, 0, (size_t)L.nb * 3 * 8));
    HIPCK(c, hipMemset(c->ws + L.o_gamma, 0, (size_t)L.nb * BN * 4));
    const size_t pb = (size_t)L.nb * c->Q * BN * store_bytes(c->storage);
    HIPCK(c, hipMemset(c->ws + L.o_pop[0], 0, pb));
    HIPCK(c, hipMemset(c->ws + L.o_pop[1], 0, pb));
    c->drag_steps[l] = 0;
  }
  if (!c->sc_all.empty()) {
    // stream-collide items carry their neighbour bricks (one scalar fetch per item)
    std::vector<ItemRec> rec(c->sc_all.size());
    for (size_t i = 0; i < rec.size(); ++i) {
      memset(&rec[i], 0, sizeof(ItemRec));
      rec[i].w = c->sc_all[i];
      const Level &L = c->lev[c->sc_all[i].level];
      for (int k = 0; k < 27; ++k) rec[i].nbr[k] = L.nbr[(size_t)c->sc_all[i].brick * 27 + k];
    }
    HIPCK(c, hipMemcpy(c->ws + c->o_sc, rec.data(), rec.size() * sizeof(ItemRec), hipMemcpyHostToDevice));
  }
  if (!c->perm_all.empty())
    HIPCK(c, hipMemcpy(c->ws + c->o_perm, c->perm_all.data(), c->perm_all.size() * sizeof(int32_t),
                       hipMemcpyHostToDevice));
  if (!c->gp_all.empty())
    HIPCK(c, hipMemcpy(c->ws + c->o_gp, c->gp_all.data(), c->gp_all.size() * sizeof(GPoint), hipMemcpyHostToDevice));
  if (!c->fine_all.empty())
    HIPCK(c, hipMemcpy(c->ws + c->o_fine, c->fine_all.data(), c->fine_all.size() * sizeof(CItem),
                       hipMemcpyHostToDevice));
  if (!c->ring_all.empty())
    HIPCK(c, hipMemcpy(c->ws + c->o_ring, c->ring_all.data(), c->ring_all.size() * sizeof(CItem),
                       hipMemcpyHostToDevice));
  if (!c->tiles_all.empty())
    HIPCK(c, hipMemcpy(c->ws + c->o_tiles, c->tiles_all.data(), c->tiles_all.size() * sizeof(CTile),
                       hipMemcpyHostToDevice));
  if (!c->tile_rows_all.empty())
    HIPCK(c, hipMemcpy(c->ws + c->o_trows, c->tile_rows_all.data(), c->tile_rows_all.size() * sizeof(int32_t),
                       hipMemcpyHostToDevice));
  if (!c->tsten_all.empty())
    HIPCK(c, hipMemcpy(c->ws + c->o_sten, c->tsten_all.data(), c->tsten_all.size() * sizeof(StencilEntry),
                       hipMemcpyHostToDevice));
  if (!c->red_items.empty())
    HIPCK(c, hipMemcpy(c->ws + c->o_redit, c->red_items.data(), c->red_items.size() * sizeof(WorkItem),
                       hipMemcpyHostToDevice));
  c->parity = 0;
  c->bound = true;
  elbm_status s = upload_static(c);
  if (s) return s;
  HIPCK(c, hipDeviceSynchronize());
  return ELBM_OK;
}

elbm_status elbm_init_fields(elbm_ctx *c, int level, const double *rho, const double *u, const double *noise) {
  if (!c || !rho || !u) return ELBM_EINVAL;
  elbm_status s = check_level(c, level);
  if (s) return s;
  if (!c->bound) FAIL(c, ELBM_ESTATE, "init before bind");
  const Level &L = c->lev[level];
  const size_t tot = (size_t)(L.bn[0] * L.bn[1] * L.bn[2]);
  const size_t nb = tot * (1 + c->D + (noise ? c->Q : 0)) * sizeof(double);
  double *d = nullptr;
  HIPCK(c, hipMalloc((void **)&d, nb));
  hipError_t e = hipMemcpy(d, rho, tot * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d + tot, u, tot * c->D * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess && noise) e = hipMemcpy(d + tot * (1 + c->D), noise, tot * c->Q * 8, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    hipFree(d);
    FAIL(c, ELBM_EDEVICE, "upload: %s", hipGetErrorString(e));
  }
  const int cur = level == 0 ? c->parity : 0;
  Dims box;
  for (int a = 0; a < 3; ++a) box.n[a] = L.bn[a];
  int rc = launch_init(c->D, c->storage, c->ws + L.o_pop[cur], (const LevelStatic *)(c->ws + c->o_levstatic), level,
                       L.nb, (const int32_t *)(c->ws + L.o_borg), box, d, d + tot,
                       noise ? d + tot * (1 + c->D) : nullptr, c->stream);
  e = hipStreamSynchronize(c->stream);
  hipFree(d);
  if (rc) FAIL(c, ELBM_EDEVICE, "init kernel: %s", hipGetErrorString((hipError_t)rc));
  if (e != hipSuccess) FAIL(c, ELBM_EDEVICE, "init: %s", hipGetErrorString(e));
  return ELBM_OK;
}

elbm_status elbm_init_fields_static(elbm_ctx *c, int level, const double *rho, const double *u,
                                    const double *noise) {
  if (!c || !rho || !u) return ELBM_EINVAL;
  elbm_status s = check_level(c, level);
  if (s) return s;
  if (!c->bound || !c->static_staging) FAIL(c, ELBM_ESTATE, "init before bind");
  const Level &L = c->lev[level];
  const size_t tot = (size_t)(L.bn[0] * L.bn[1] * L.bn[2]);
  const size_t nb = tot * (1 + c->D + (noise ? c->Q : 0)) * sizeof(double);
  if (nb > kStaticStagingBytes)
    FAIL(c, ELBM_EINVAL, "level %d needs %zu bytes of staging, more than the %zu of the static buffer", level, nb,
         kStaticStagingBytes);
  // the staging copies follow the work already enqueued on the bound stream (an earlier
  // call's init kernel may still read the buffer)
  double *d = (double *)c->static_staging;
  HIPCK(c, hipMemcpyAsync(d, rho, tot * 8, hipMemcpyHostToDevice, c->stream));
  HIPCK(c, hipMemcpyAsync(d + tot, u, tot * c->D * 8, hipMemcpyHostToDevice, c->stream));
  if (noise) HIPCK(c, hipMemcpyAsync(d + tot * (1 + c->D), noise, tot * c->Q * 8, hipMemcpyHostToDevice, c->stream));
  const int cur = level == 0 ? c->parity : 0;
  Dims box;
  for (int a = 0; a < 3; ++a) box.n[a] = L.bn[a];
  LCK(c, launch_init(c->D, c->storage, c->ws + L.o_pop[cur], (const LevelStatic *)(c->ws + c->o_levstatic), level,
                     L.nb, (const int32_t *)(c->ws + L.o_borg), box, d, d + tot,
                     noise ? d + tot * (1 + c->D) : nullptr, c->stream));
  HIPCK(c, hipStreamSynchronize(c->stream));
  return ELBM_OK;
}

elbm_status elbm_set_force_field(elbm_ctx *c, int level, const double *F) {
  if (!c) return ELBM_EINVAL;
  elbm_status s = check_level(c, level);
  if (s) return s;
  if (!c->bound) FAIL(c, ELBM_ESTATE, "set_force_field before bind");
  Level &L = c->lev[level];
  const bool was = L.force_on;
  if (F) {
    Dims box;
    for (int a = 0; a < 3; ++a) box.n[a] = L.bn[a];
    LCK(c, launch_force_scatter(c->D, (float *)(c->ws + L.o_force), F, L.nb, (const int32_t *)(c->ws + L.o_borg),
                                box, c->stream));
    L.force_on = true;
  } else {
    L.force_on = false;
  }
  if (was != L.force_on) {
    HIPCK(c, hipStreamSynchronize(c->stream));
    s = upload_static(c);
    if (s) return s;
    invalidate_graphs(c);
  }
  return ELBM_OK;
}

elbm_status elbm_advance(elbm_ctx *c, int n) {
  if (!c) return ELBM_EINVAL;
  if (!c->bound) FAIL(c, ELBM_ESTATE, "advance before bind");
  if (n < 0) FAIL(c, ELBM_EINVAL, "negative step count");
  if (c->use_graph && !c->timing && !c->graph_valid) {
    elbm_status s = build_graphs(c);
    if (s) return s;
  }
  // whole multi-step graphs first, then single steps
  const int G = (c->use_graph > 1 && !c->timing) ? c->use_graph : 1;
  for (; G > 1 && n >= G; n -= G) {
    HIPCK(c, hipGraphLaunch(c->graphm[c->parity], c->stream));
    c->parity ^= G & 1;
    for (int l = 0; l < c->L; ++l) c->drag_steps[l] += (int64_t)G << l;
  }
  for (int i = 0; i < n; ++i) {
    if (c->use_graph && !c->timing) {
      HIPCK(c, hipGraphLaunch(c->graph[c->parity], c->stream));
    } else {
      elbm_status s = enqueue_coarse_step(c, c->parity, c->stream, c->side, false);
      if (s) return s;
    }
    c->parity ^= 1;
    for (int l = 0; l < c->L; ++l) c->drag_steps[l] += (int64_t)1 << l;
  }
  return ELBM_OK;
}

elbm_status elbm_read_moments(elbm_ctx *c, int level, double *rho, double *u, double *gamma) {
  if (!c) return ELBM_EINVAL;
  elbm_status s = check_level(c, level);
  if (s) return s;
  if (!c->bound) FAIL(c, ELBM_ESTATE, "read before bind");
  const Level &L = c->lev[level];
  Dims box;
  for (int a = 0; a < 3; ++a) box.n[a] = L.bn[a];
  const size_t tot = (size_t)(L.bn[0] * L.bn[1] * L.bn[2]);
  if (rho) LCK(c, launch_fill_nan(rho, tot, c->stream));
  if (u) LCK(c, launch_fill_nan(u, tot * c->D, c->stream));
  if (gamma) LCK(c, launch_fill_nan(gamma, tot, c->stream));
  const int cur = level == 0 ? c->parity : 0;
  LCK(c, launch_read(c->D, c->storage, c->ws + L.o_pop[cur], (const LevelStatic *)(c->ws + c->o_levstatic), level,
                     L.nb, (const int32_t *)(c->ws + L.o_borg), box, rho, u, gamma, nullptr, c->stream));
  return ELBM_OK;
}

// ---------------------------------------------------------------- re-meshing
// Transfer of the current state onto a lattice with other refinement blocks (the
// adaptive refinement the conclusion, Sec. V, proposes).  The host decides where every
// node of the new lattice takes its state from; remesh.hip does the arithmetic.
namespace {
// post-collision non-equilibrium factor from level lc to level lc + 1
double post_factor(const elbm_ctx *c, int lc) {
  const double bc = c->lev[lc].beta, bf = c->lev[lc + 1].beta;
  return bc * (1.0 - 2.0 * bf) / (2.0 * bf * (1.0 - 2.0 * bc));
}
// a fluid node of level l at position x, or brick -1
NodeRef fluid_at(const elbm_ctx *c, int l, const int64_t x[3]) {
  NodeRef r = locate(c, l, x);
  if (r.brick >= 0 && c->lev[l].solid[(size_t)r.brick * BN + r.node]) r.brick = -2;
  return r;
}
}  // namespace

elbm_status elbm_transfer_state(elbm_ctx *d, const elbm_ctx *s) {
  if (!d || !s || d == s) return ELBM_EINVAL;
  if (!d->bound || !s->bound) FAIL(d, ELBM_ESTATE, "transfer between lattices that are not both bound");
  bool same = d->D == s->D && d->storage == s->storage && d->L == s->L && d->nu0 == s->nu0;
  for (int a = 0; a < 3; ++a) same = same && d->N[a] == s->N[a] && d->periodic[a] == s->periodic[a] && d->Fu[a] == s->Fu[a];
  for (int f = 0; f < 6; ++f) {
    same = same && d->face_kind[f] == s->face_kind[f];
    for (int a = 0; a < 3; ++a) same = same && d->face_u[f][a] == s->face_u[f][a];
  }
  if (!same) FAIL(d, ELBM_EINVAL, "transfer: the lattices differ in domain, levels, storage, parameters or boundaries");
  std::vector<TPoint> pts;
  std::unordered_map<int64_t, int32_t> pidx;
  std::vector<TItem> items;
  std::vector<StencilEntry> sten;
  auto point = [&](int level, NodeRef r, double fac, int parent) -> int32_t {
    const int64_t key = ((int64_t)(level * 2 + parent) << 48) | ((int64_t)r.brick << 8) | (int64_t)r.node;
    auto it = pidx.find(key);
    if (it != pidx.end()) return it->second;
    TPoint p;
    p.brick = r.brick;
    p.node = (uint16_t)r.node;
    p.level = (uint8_t)level;
    p.pad = 0;
    p.fac = fac;
    pts.push_back(p);
    pidx.emplace(key, (int32_t)pts.size() - 1);
    return (int32_t)pts.size() - 1;
  };
  static const float w4[4] = {-1.0f / 16.0f, 9.0f / 16.0f, 9.0f / 16.0f, -1.0f / 16.0f};
  for (int l = 0; l < d->L; ++l) {
    const Level &L = d->lev[l];
    for (int32_t b = 0; b < L.nb; ++b)
      for (int n = 0; n < BN; ++n) {
        const size_t k = (size_t)b * BN + n;
        if (!L.exists[k] || L.solid[k]) continue;
        int64_t x[3] = {0, 0, 0};
        int rem = n;
        for (int a = 0; a < 3; ++a) {
          const int bd = bdim(d->D, a);
          x[a] = L.blo[a] + L.borg[(size_t)b * 3 + a] + rem % bd;
          rem /= bd;
        }
        TItem it;
        it.brick = b;
        it.node = (uint16_t)n;
        it.level = (uint8_t)l;
        NodeRef r = fluid_at(s, l, x);
        if (r.brick == -2) FAIL(d, ELBM_EINVAL, "transfer: a level %d fluid node is solid in the old lattice", l);
        if (r.brick >= 0) {
          it.kind = 0;
          it.a = r.brick;
          it.b = r.node;
          items.push_back(it);
          continue;
        }
        if (l + 1 < d->L) {
          const int64_t xc[3] = {2 * x[0], 2 * x[1], 2 * x[2]};
          NodeRef rc = fluid_at(s, l + 1, xc);
          if (rc.brick >= 0) {
            it.kind = 1;
            it.a = rc.brick;
            it.b = rc.node;
            items.push_back(it);
            continue;
          }
        }
        if (l == 0) FAIL(d, ELBM_EINVAL, "transfer: no old value for a level 0 node");
        // four-point reconstruction over the axes where x is not on a parent node
        int npt[3] = {1, 1, 1};
        int64_t P[3][4];
        float W[3][4];
        for (int a = 0; a < 3; ++a) {
          if (a < d->D && (x[a] & 1)) {
            npt[a] = 4;
            for (int q = 0; q < 4; ++q) {
              P[a][q] = (x[a] - 3 + 2 * q) / 2;
              W[a][q] = w4[q];
            }
          } else {
            P[a][0] = x[a] / 2;
            W[a][0] = 1.0f;
          }
        }
        it.kind = 2;
        it.a = (int32_t)sten.size();
        for (int kz = 0; kz < npt[2]; ++kz)
          for (int ky = 0; ky < npt[1]; ++ky)
            for (int kx = 0; kx < npt[0]; ++kx) {
              const int64_t X[3] = {P[0][kx], P[1][ky], P[2][kz]};
              const int64_t xf[3] = {2 * X[0], 2 * X[1], 2 * X[2]};
              NodeRef rf = fluid_at(s, l, xf);
              int32_t slot;
              if (rf.brick >= 0) {
                slot = point(l, rf, 1.0, 0);
              } else {
                NodeRef rp = fluid_at(s, l - 1, X);
                if (rp.brick < 0)
                  FAIL(d, ELBM_EINVAL, "transfer: level %d node (%lld,%lld,%lld) has no old value to reconstruct from", l,
                       (long long)x[0], (long long)x[1], (long long)x[2]);
                slot = point(l - 1, rp, post_factor(s, l - 1), 1);
              }
              StencilEntry e;
              e.slot = slot;
              e.w = W[0][kx] * W[1][ky] * W[2][kz];
              sten.push_back(e);
            }
        it.b = (int32_t)sten.size() - it.a;
        items.push_back(it);
      }
  }
  // device copies of the tables and the staged rows (a transfer is rare: allocated
  // here and released before returning)
  const size_t row_bytes = (size_t)stage_row_width(d->D) * comp_bytes(d->storage);
  const size_t o_pts = 0, o_items = align_up(o_pts + pts.size() * sizeof(TPoint) + 1, 256),
               o_sten = align_up(o_items + items.size() * sizeof(TItem) + 1, 256),
               o_stage = align_up(o_sten + sten.size() * sizeof(StencilEntry) + 1, 256),
               total = o_stage + std::max<size_t>(pts.size(), 1) * row_bytes;
  HIPCK(d, hipStreamSynchronize(s->stream));  // the old state is complete
  char *buf = nullptr;
  HIPCK(d, hipMalloc((void **)&buf, total));
  hipError_t e = hipSuccess;
  if (!pts.empty()) e = hipMemcpy(buf + o_pts, pts.data(), pts.size() * sizeof(TPoint), hipMemcpyHostToDevice);
  if (e == hipSuccess && !items.empty())
    e = hipMemcpy(buf + o_items, items.data(), items.size() * sizeof(TItem), hipMemcpyHostToDevice);
  if (e == hipSuccess && !sten.empty())
    e = hipMemcpy(buf + o_sten, sten.data(), sten.size() * sizeof(StencilEntry), hipMemcpyHostToDevice);
  TransferArgs a;
  memset(&a, 0, sizeof(a));
  a.pts = (const TPoint *)(buf + o_pts);
  a.n_pts = (int)pts.size();
  a.items = (const TItem *)(buf + o_items);
  a.n_items = (int)items.size();
  a.sten = (const StencilEntry *)(buf + o_sten);
  a.stage = buf + o_stage;
  for (int l = 0; l < d->L; ++l) {
    a.src[l] = s->ws + s->lev[l].o_pop[l == 0 ? s->parity : 0];
    a.dst[l] = d->ws + d->lev[l].o_pop[l == 0 ? d->parity : 0];
    a.fac_coal[l] = l + 1 < d->L ? 1.0 / post_factor(s, l) : 1.0;
  }
  int rc = 0;
  if (e == hipSuccess) rc = launch_transfer(d->D, d->storage, a, d->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(d->stream);
  hipFree(buf);
  if (rc) FAIL(d, ELBM_EDEVICE, "transfer kernels: %s", hipGetErrorString((hipError_t)rc));
  if (e != hipSuccess) FAIL(d, ELBM_EDEVICE, "transfer: %s", hipGetErrorString(e));
  for (int l = 0; l < d->L; ++l) {
    LCK(d, launch_zero(d->ws + d->lev[l].o_drag, (size_t)d->lev[l].nb * 3 * 8, d->stream));
    d->drag_steps[l] = 0;
  }
  HIPCK(d, hipStreamSynchronize(d->stream));
  return ELBM_OK;
}

elbm_status elbm_stream_copy(void *dst, const void *src, size_t bytes, int grid, void *stream) {
  if (!dst || !src || (bytes & 15) || grid < 0) return ELBM_EINVAL;
  if (grid == 0) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    grid = 4 * (cus > 0 ? cus : 256);
  }
  return launch_stream_copy(dst, src, bytes, grid, stream) ? ELBM_EDEVICE : ELBM_OK;
}

elbm_status elbm_brick_dims(int D, int64_t dims[3]) {
  if ((D != 2 && D != 3) || !dims) return ELBM_EINVAL;
  for (int a = 0; a < 3; ++a) dims[a] = bdim(D, a);
  return ELBM_OK;
}

elbm_status elbm_gamma_indicator(elbm_ctx *c, int level, float *out, int64_t grid[3]) {
  if (!c || !grid) return ELBM_EINVAL;
  elbm_status s = check_level(c, level);
  if (s) return s;
  const Level &L = c->lev[level];
  for (int a = 0; a < 3; ++a) grid[a] = L.gdim[a];
  if (!out) return ELBM_OK;
  if (!c->bound) FAIL(c, ELBM_ESTATE, "indicator before bind");
  if (!c->gamma_on) FAIL(c, ELBM_ESTATE, "the indicator reads the per-node gamma: enable elbm_set_gamma_output first");
  Dims box, g;
  for (int a = 0; a < 3; ++a) {
    box.n[a] = L.bn[a];
    g.n[a] = L.gdim[a];
  }
  LCK(c, launch_gamma_indicator(c->D, (const LevelStatic *)(c->ws + c->o_levstatic), level, L.nb,
                                (const int32_t *)(c->ws + L.o_borg), box, g, out, c->stream));
  return ELBM_OK;
}

elbm_status elbm_read_populations(elbm_ctx *c, int level, double *f) {
  if (!c || !f) return ELBM_EINVAL;
  elbm_status s = check_level(c, level);
  if (s) return s;
  if (!c->bound) FAIL(c, ELBM_ESTATE, "read before bind");
  const Level &L = c->lev[level];
  Dims box;
  for (int a = 0; a < 3; ++a) box.n[a] = L.bn[a];
  const size_t tot = (size_t)(L.bn[0] * L.bn[1] * L.bn[2]);
  LCK(c, launch_fill_nan(f, tot * c->Q, c->stream));
  const int cur = level == 0 ? c->parity : 0;
  LCK(c, launch_read(c->D, c->storage, c->ws + L.o_pop[cur], (const LevelStatic *)(c->ws + c->o_levstatic), level,
                     L.nb, (const int32_t *)(c->ws + L.o_borg), box, nullptr, nullptr, nullptr, f, c->stream));
  return ELBM_OK;
}

elbm_status elbm_sample_populations(elbm_ctx *c, int level, int64_t n, const int64_t *coords, double *out) {
  if (!c || (n > 0 && (!coords || !out)) || n < 0) return ELBM_EINVAL;
  elbm_status s = check_level(c, level);
  if (s) return s;
  if (!c->bound) FAIL(c, ELBM_ESTATE, "sample before bind");
  const Level &L = c->lev[level];
  const int cur = level == 0 ? c->parity : 0;
  const int64_t chunk = (int64_t)((c->tmp_bytes - 512) / (8 + 8 * c->Q));
  std::vector<int32_t> br, nd;
  for (int64_t s0 = 0; s0 < n; s0 += chunk) {
    const int64_t m = std::min(chunk, n - s0);
    br.assign((size_t)m, -1);
    nd.assign((size_t)m, 0);
    for (int64_t i = 0; i < m; ++i) {
      NodeRef r = locate(c, level, coords + 3 * (s0 + i));
      if (r.brick >= 0 && !L.solid[(size_t)r.brick * BN + r.node]) {
        br[i] = r.brick;
        nd[i] = r.node;
      }
    }
    char *tmp = c->ws + c->o_tmp;
    HIPCK(c, hipMemcpyAsync(tmp, br.data(), m * 4, hipMemcpyHostToDevice, c->stream));
    HIPCK(c, hipMemcpyAsync(tmp + m * 4, nd.data(), m * 4, hipMemcpyHostToDevice, c->stream));
    double *dout = (double *)(tmp + align_up(m * 8, 256));
    LCK(c, launch_sample(c->D, c->storage, c->ws + L.o_pop[cur], nullptr, level, (int)m, (const int32_t *)tmp,
                         (const int32_t *)(tmp + m * 4), dout, c->stream));
    HIPCK(c, hipMemcpyAsync(out + s0 * c->Q, dout, m * c->Q * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCK(c, hipStreamSynchronize(c->stream));
  }
  return ELBM_OK;
}

elbm_status elbm_reduce(elbm_ctx *c, double *mass, double mom[3], int64_t *n_unstable) {
  if (!c) return ELBM_EINVAL;
  if (!c->bound) FAIL(c, ELBM_ESTATE, "reduce before bind");
  void *pops[MAXL] = {};
  for (int l = 0; l < c->L; ++l) pops[l] = c->ws + c->lev[l].o_pop[l == 0 ? c->parity : 0];
  LCK(c, launch_reduce(c->D, c->storage, pops, (const LevelStatic *)(c->ws + c->o_levstatic),
                       (const WorkItem *)(c->ws + c->o_redit), (int)c->red_items.size(), (double *)(c->ws + c->o_part),
                       (double *)(c->ws + c->o_res), c->stream));
  double r[5];
  HIPCK(c, hipMemcpyAsync(r, c->ws + c->o_res, sizeof(r), hipMemcpyDeviceToHost, c->stream));
  HIPCK(c, hipStreamSynchronize(c->stream));
  double vol = 0;
  for (int l = 0; l < c->L; ++l)
    for (float w : c->lev[l].weight) vol += w;
  if (mass) *mass = vol + r[0];
  if (mom)
    for (int a = 0; a < 3; ++a) mom[a] = a < c->D ? r[1 + a] : 0.0;
  if (n_unstable) *n_unstable = (int64_t)llround(r[4]);
  return ELBM_OK;
}

elbm_status elbm_check(elbm_ctx *c) {
  int64_t bad = 0;
  double m, j[3];
  elbm_status s = elbm_reduce(c, &m, j, &bad);
  if (s) return s;
  if (bad > 0 || !std::isfinite(m)) FAIL(c, ELBM_EUNSTABLE, "%lld unstable nodes", (long long)bad);
  return ELBM_OK;
}

elbm_status elbm_drag(elbm_ctx *c, int level, double F[3], int64_t *steps, int reset) {
  if (!c || !F) return ELBM_EINVAL;
  elbm_status s = check_level(c, level);
  if (s) return s;
  if (!c->bound) FAIL(c, ELBM_ESTATE, "drag before bind");
  const Level &L = c->lev[level];
  std::vector<double> part((size_t)L.nb * 3);
  HIPCK(c, hipMemcpyAsync(part.data(), c->ws + L.o_drag, part.size() * 8, hipMemcpyDeviceToHost, c->stream));
  HIPCK(c, hipStreamSynchronize(c->stream));
  double acc[3] = {0, 0, 0};
  for (int32_t b = 0; b < L.nb; ++b)
    for (int a = 0; a < 3; ++a) acc[a] += part[(size_t)b * 3 + a];
  for (int a = 0; a < 3; ++a) F[a] = acc[a];
  if (steps) *steps = c->drag_steps[level];
  if (reset) {
    LCK(c, launch_zero(c->ws + L.o_drag, (size_t)L.nb * 3 * 8, c->stream));
    HIPCK(c, hipStreamSynchronize(c->stream));
    c->drag_steps[level] = 0;
  }
  return ELBM_OK;
}

elbm_status elbm_set_gamma_output(elbm_ctx *c, int enable) {
  if (!c) return ELBM_EINVAL;
  c->gamma_on = enable != 0;
  if (c->bound) {
    elbm_status s = upload_static(c);
    if (s) return s;
    invalidate_graphs(c);
  }
  return ELBM_OK;
}

elbm_status elbm_set_launch(elbm_ctx *c, int use_graph, int wg_per_cu, int xcd_remap, int threads, int occupancy,
                            int pipeline) {
  if (!c) return ELBM_EINVAL;
  if (occupancy != 1 && occupancy != 4) FAIL(c, ELBM_EINVAL, "occupancy variant must be 1 or 4");
  if (threads != 64 && threads != 128 && threads != 256) FAIL(c, ELBM_EINVAL, "threads must be 64, 128 or 256");
  if (wg_per_cu < 0 || wg_per_cu > 64) FAIL(c, ELBM_EINVAL, "wg_per_cu out of range");
  if (pipeline < 0 || pipeline > 2) FAIL(c, ELBM_EINVAL, "pipeline must be 0, 1 or 2");
  if (use_graph < 0 || use_graph > 64) FAIL(c, ELBM_EINVAL, "use_graph must be 0..64");
  if (xcd_remap < 0 || xcd_remap > 4096) FAIL(c, ELBM_EINVAL, "xcd_remap out of range");
  c->use_graph = use_graph;
  c->wg_per_cu = wg_per_cu;
  c->xcd_remap = xcd_remap;
  c->threads = threads;
  c->occ = occupancy;
  c->pipe = pipeline;
  invalidate_graphs(c);
  return ELBM_OK;
}

elbm_status elbm_get_launch(const elbm_ctx *c, int32_t cfg[6]) {
  if (!c || !cfg) return ELBM_EINVAL;
  cfg[0] = c->use_graph;
  cfg[1] = c->wg_per_cu;
  cfg[2] = c->xcd_remap;
  cfg[3] = c->threads;
  cfg[4] = c->occ;
  cfg[5] = c->pipe;
  return ELBM_OK;
}

elbm_status elbm_synchronize(elbm_ctx *c) {
  if (!c) return ELBM_EINVAL;
  HIPCK(c, hipStreamSynchronize(c->stream));
  return ELBM_OK;
}

elbm_status elbm_profile(elbm_ctx *c, int steps, double *ms_total, double *ms_sc, int64_t *n_launch) {
  if (!c) return ELBM_EINVAL;
  if (!c->bound) FAIL(c, ELBM_ESTATE, "profile before bind");
  for (hipEvent_t e : c->tev) hipEventDestroy(e);
  c->tev.clear();
  hipEvent_t a, b;
  HIPCK(c, hipEventCreate(&a));
  HIPCK(c, hipEventCreate(&b));
  c->timing = true;
  HIPCK(c, hipEventRecord(a, c->stream));
  elbm_status s = elbm_advance(c, steps);
  hipError_t e = hipEventRecord(b, c->stream);
  c->timing = false;
  if (s) return s;
  if (e != hipSuccess) FAIL(c, ELBM_EDEVICE, "event record: %s", hipGetErrorString(e));
  HIPCK(c, hipEventSynchronize(b));
  float tot = 0;
  HIPCK(c, hipEventElapsedTime(&tot, a, b));
  double sc = 0;
  for (size_t i = 0; i + 1 < c->tev.size(); i += 2) {
    float m = 0;
    HIPCK(c, hipEventElapsedTime(&m, c->tev[i], c->tev[i + 1]));
    sc += m;
  }
  if (ms_total) *ms_total = tot;
  if (ms_sc) *ms_sc = sc;
  if (n_launch) *n_launch = (int64_t)(c->tev.size() / 2);
  for (hipEvent_t ev : c->tev) hipEventDestroy(ev);
  c->tev.clear();
  hipEventDestroy(a);
  hipEventDestroy(b);
  return ELBM_OK;
}

elbm_status elbm_state_bytes(const elbm_ctx *c, size_t *bytes) {
  if (!c || !bytes) return ELBM_EINVAL;
  if (!c->finalized) return ELBM_ESTATE;
  size_t t = 0;
  for (int l = 0; l < c->L; ++l) t += (size_t)c->lev[l].nb * c->Q * BN * store_bytes(c->storage);
  *bytes = t;
  return ELBM_OK;
}

elbm_status elbm_save_state(elbm_ctx *c, void *dst) {
  if (!c || !dst) return ELBM_EINVAL;
  if (!c->bound) FAIL(c, ELBM_ESTATE, "save before bind");
  size_t off = 0;
  for (int l = 0; l < c->L; ++l) {
    const Level &L = c->lev[l];
    const size_t pb = (size_t)L.nb * c->Q * BN * store_bytes(c->storage);
    LCK(c, launch_copy((char *)dst + off, c->ws + L.o_pop[l == 0 ? c->parity : 0], pb, c->stream));
    off += pb;
  }
  return ELBM_OK;
}

elbm_status elbm_load_state(elbm_ctx *c, const void *src) {
  if (!c || !src) return ELBM_EINVAL;
  if (!c->bound) FAIL(c, ELBM_ESTATE, "load before bind");
  size_t off = 0;
  for (int l = 0; l < c->L; ++l) {
    const Level &L = c->lev[l];
    const size_t pb = (size_t)L.nb * c->Q * BN * store_bytes(c->storage);
    LCK(c, launch_copy(c->ws + L.o_pop[l == 0 ? c->parity : 0], (const char *)src + off, pb, c->stream));
    off += pb;
  }
  return ELBM_OK;
}


elbm_status elbm_tune(elbm_ctx *c, const char *cache_path, int steps) {
  (void)steps;
  if (!c) return ELBM_EINVAL;
  if (!c->bound) FAIL(c, ELBM_ESTATE, "tune before bind");
  // cache key: dimension, storage and bricks per level
  std::string key = "d" + std::to_string(c->D) + "s" + std::to_string(c->storage);
  for (int l = 0; l < c->L; ++l) key += "_" + std::to_string(c->lev[l].nb);
  if (cache_path) {
    FILE *f = fopen(cache_path, "r");
    if (f) {
      char line[512];
      while (fgets(line, sizeof(line), f)) {
        char k[256];
        int g, w, x, t, o, p;
        if (sscanf(line, " \"%255[^\"]\": [%d, %d, %d, %d, %d, %d]", k, &g, &w, &x, &t, &o, &p) == 7 && key == k) {
          fclose(f);
          return elbm_set_launch(c, g, w, x, t, o, p);
        }
      }
      fclose(f);
    }
  }
  // No search runs here: launch configurations are timed by paper_1608_06915_amd/tune.py,
  // each candidate in a process of its own, which writes the cache read above.  (An
  // in-process search that captured, instantiated and destroyed two graphs per candidate
  // twice ended its process with a host segmentation fault whose cause was not found.)
  FAIL(c, ELBM_ESTATE, "no cached launch configuration for %s", key.c_str());
}


// ---------------------------------------------------------------- discrete adjoint
elbm_status elbm_adjoint_bytes(elbm_ctx *c, int n_max, int K, size_t *bytes) {
  if (!c || !bytes) return ELBM_EINVAL;
  if (!c->finalized) FAIL(c, ELBM_ESTATE, "adjoint_bytes before finalize");
  if (n_max < 1 || K < 1) FAIL(c, ELBM_EINVAL, "adjoint: need n_max >= 1 and K >= 1");
  adj_build_tables(c);
  adj_layout(c, n_max, K);
  *bytes = c->adj.need;
  return ELBM_OK;
}

elbm_status elbm_adjoint_bind(elbm_ctx *c, void *ws, size_t bytes, int n_max, int K) {
  if (!c || !ws) return ELBM_EINVAL;
  if (!c->bound) FAIL(c, ELBM_ESTATE, "adjoint_bind before bind");
  if (n_max < 1 || K < 1) FAIL(c, ELBM_EINVAL, "adjoint: need n_max >= 1 and K >= 1");
  if ((uintptr_t)ws & 255) FAIL(c, ELBM_EINVAL, "adjoint workspace must be 256-byte aligned");
  auto &A = c->adj;
  adj_build_tables(c);
  adj_layout(c, n_max, K);
  if (bytes < A.need) FAIL(c, ELBM_ESMALL, "adjoint workspace %zu bytes < %zu required", bytes, A.need);
  A.ws = (char *)ws;
  A.nmax = n_max;
  A.K = K;
  A.pending = false;
  A.n = 0;
  const size_t tb = comp_bytes(c->storage);
  AdjLevel al[MAXL];
  memset(al, 0, sizeof(al));
  for (int l = 0; l < c->L; ++l) {
    const size_t nb = (size_t)c->lev[l].nb;
    al[l].zero_brick = (int32_t)nb;
    if (A.has_amask[l]) {
      al[l].amask = (const uint32_t *)(A.ws + A.o_amask[l]);
      HIPCK(c, hipMemcpy(A.ws + A.o_amask[l], A.amask[l].data(), A.amask[l].size() * 4, hipMemcpyHostToDevice));
    }
    LCK(c, launch_zero(A.ws + A.o_lg[l][0], (nb + 1) * c->Q * BN * tb, c->stream));
    LCK(c, launch_zero(A.ws + A.o_lg[l][1], (nb + 1) * c->Q * BN * tb, c->stream));
    LCK(c, launch_zero(A.ws + A.o_lam[l][0], nb * c->Q * BN * tb, c->stream));
    LCK(c, launch_zero(A.ws + A.o_lam[l][1], nb * c->Q * BN * tb, c->stream));
    LCK(c, launch_zero(A.ws + A.o_lF[l], nb * c->D * BN * tb, c->stream));
  }
  HIPCK(c, hipStreamSynchronize(c->stream));
  HIPCK(c, hipMemcpy(A.ws + A.o_alev, al, sizeof(al), hipMemcpyHostToDevice));
  if (!A.tofs.empty()) HIPCK(c, hipMemcpy(A.ws + A.o_tofs, A.tofs.data(), A.tofs.size() * 4, hipMemcpyHostToDevice));
  if (!A.tsten.empty())
    HIPCK(c, hipMemcpy(A.ws + A.o_tsten, A.tsten.data(), A.tsten.size() * sizeof(StencilEntry),
                       hipMemcpyHostToDevice));
  if (!A.items.empty())
    HIPCK(c, hipMemcpy(A.ws + A.o_items, A.items.data(), A.items.size() * sizeof(WorkItem), hipMemcpyHostToDevice));
  if (!A.bitems.empty())
    HIPCK(c, hipMemcpy(A.ws + A.o_bitems, A.bitems.data(), A.bitems.size() * sizeof(WorkItem), hipMemcpyHostToDevice));
  A.bound = true;
  return ELBM_OK;
}

elbm_status elbm_adjoint_forward(elbm_ctx *c, int n, int objective, int body_level, const double dir[3],
                                 double *J) {
  if (!c) return ELBM_EINVAL;
  auto &A = c->adj;
  if (!A.bound) FAIL(c, ELBM_ESTATE, "adjoint_forward before adjoint_bind");
  if (n < 1 || n > A.nmax) FAIL(c, ELBM_EINVAL, "adjoint: step count %d outside 1..%d", n, A.nmax);
  if (objective != ELBM_OBJ_DRAG && objective != ELBM_OBJ_KE) FAIL(c, ELBM_EINVAL, "unknown objective %d", objective);
  if (objective == ELBM_OBJ_DRAG) {
    if (body_level < 0 || body_level >= c->L) FAIL(c, ELBM_EINVAL, "bad body level %d", body_level);
    if (!dir) FAIL(c, ELBM_EINVAL, "drag objective needs a direction");
  }
  A.pending = false;
  A.n = n;
  A.objective = objective;
  A.body_level = objective == ELBM_OBJ_DRAG ? body_level : -1;
  for (int q = 0; q < 3; ++q) A.dir[q] = (objective == ELBM_OBJ_DRAG) ? dir[q] : 0.0;
  const size_t tb = comp_bytes(c->storage);
  for (int l = 0; l < c->L; ++l) LCK(c, launch_zero(A.ws + A.o_lF[l], (size_t)c->lev[l].nb * c->D * BN * tb, c->stream));
  if (objective == ELBM_OBJ_DRAG) {
    LCK(c, launch_zero(c->ws + c->lev[body_level].o_drag, (size_t)c->lev[body_level].nb * 3 * 8, c->stream));
    c->drag_steps[body_level] = 0;
  }
  hipEvent_t e0, e1;
  HIPCK(c, hipEventCreate(&e0));
  HIPCK(c, hipEventCreate(&e1));
  HIPCK(c, hipEventRecord(e0, c->stream));
  const int S = (n + A.K - 1) / A.K;
  for (int s = 0; s < S; ++s) {
    for (int l = 0; l < c->L; ++l) LCK(c, launch_copy(adj_ckpt(c, s, l), cur_state(c, l), level_state_bytes(c, l), c->stream));
    elbm_status st = elbm_advance(c, std::min(A.K, n - s * A.K));
    if (st) return st;
  }
  HIPCK(c, hipEventRecord(e1, c->stream));
  double val = 0;
  if (objective == ELBM_OBJ_DRAG) {
    double F[3];
    int64_t steps = 0;
    elbm_status st = elbm_drag(c, body_level, F, &steps, 1);
    if (st) return st;
    val = (F[0] * dir[0] + F[1] * dir[1] + F[2] * dir[2]) / (double)(steps > 0 ? steps : 1);
    for (int l = 0; l < c->L; ++l)
      LCK(c, launch_zero(A.ws + A.o_lam[l][0], (size_t)c->lev[l].nb * c->Q * BN * tb, c->stream));
  } else {
    AdjKEArgs k;
    memset(&k, 0, sizeof(k));
    k.items = (const WorkItem *)(c->ws + c->o_redit);
    k.n_items = (int)c->red_items.size();
    k.lev = (const LevelStatic *)(c->ws + c->o_levstatic);
    for (int l = 0; l < c->L; ++l) {
      k.pop[l] = cur_state(c, l);
      k.lam[l] = A.ws + A.o_lam[l][0];
      k.lF[l] = A.ws + A.o_lF[l];
    }
    k.partials = (double *)(A.ws + A.o_part);
    LCK(c, launch_adj_ke(c->D, c->storage, k, (double *)(A.ws + A.o_res), c->stream));
    HIPCK(c, hipMemcpyAsync(&val, A.ws + A.o_res, 8, hipMemcpyDeviceToHost, c->stream));
  }
  HIPCK(c, hipStreamSynchronize(c->stream));
  float ms = 0;
  HIPCK(c, hipEventElapsedTime(&ms, e0, e1));
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  A.ms[0] = ms;
  for (int l = 0; l < c->L; ++l) A.cur[l] = A.lgc[l] = 0;
  A.J = val;
  if (J) *J = val;
  A.pending = true;
  return ELBM_OK;
}

// Recompute segment s from its checkpoint into tape set s & 1 (every level substep's
// state and the staged rows of every coupling tick), on stream st.
elbm_status adj_recompute(elbm_ctx *c, int s, hipStream_t st) {
  auto &A = c->adj;
  const int T = 1 << (c->L - 1);
  const int q = s & 1;
  const int Ks = std::min(A.K, A.n - s * A.K);
  for (int l = 0; l < c->L; ++l)
    LCK(c, launch_copy(adj_tape(c, q, l, 0), adj_ckpt(c, s, l), level_state_bytes(c, l), st));
  for (int k = 1; k <= Ks; ++k)
    for (int t = 1; t <= T; ++t) {
      void *src[MAXL] = {}, *dst[MAXL] = {};
      for (int l = c->ticks[t - 1].lmin; l < c->L; ++l) {
        const size_t slot = ((size_t)(k - 1) << l) + (size_t)((t >> (c->L - 1 - l)) - 1);
        src[l] = adj_tape(c, q, l, slot);
        dst[l] = adj_tape(c, q, l, slot + 1);
      }
      elbm_status e = enqueue_tick_io(c, t, src, dst, st, c->side, false, 0,
                                      A.ctick[(size_t)t - 1] >= 0 ? adj_stage(c, q, k, t) : nullptr);
      if (e) return e;
    }
  return ELBM_OK;
}

// Segments are reversed from the last to the first.  The recomputation of segment s-1
// (tape set (s-1) & 1, on a stream of its own) runs while the reverse sweep of segment s
// reads set s & 1 on the bound stream; it waits for the reverse sweep of segment s+1,
// the last reader of its set.  Every kernel of this workload is short, so the two
// streams are fed by two host threads: a second thread enqueues the recomputations,
// and each thread waits on the host until the other has recorded the event it depends
// on before enqueueing the wait for it.
elbm_status elbm_adjoint_backward(elbm_ctx *c) {
  if (!c) return ELBM_EINVAL;
  auto &A = c->adj;
  if (!A.bound || !A.pending) FAIL(c, ELBM_ESTATE, "adjoint_backward without a preceding adjoint_forward");
  const int T = 1 << (c->L - 1);
  const int S = (A.n + A.K - 1) / A.K;
  hipStream_t R = c->side;  // idle outside graph capture and forked eager launches
  // per segment: recompute start/end (stream R), reverse start/end (bound stream); and
  // the start and end of the whole backward pass
  std::vector<hipEvent_t> ev((size_t)4 * S + 2);
  for (auto &e : ev) HIPCK(c, hipEventCreate(&e));
  auto E = [&](int s, int k) { return ev[(size_t)4 * s + k]; };
  hipEvent_t e_begin = ev[(size_t)4 * S], e_end = ev[(size_t)4 * S + 1];
  HIPCK(c, hipEventRecord(e_begin, c->stream));
  std::mutex mu;
  std::condition_variable cv;
  int rec_done = S, rev_done = S;  // lowest segment whose end event each thread has recorded
  bool stop = false;
  elbm_status pst = ELBM_OK;
  std::string perr;
  std::thread producer([&]() {
    hipError_t e = hipStreamWaitEvent(R, e_begin, 0);  // after everything before this call
    for (int s = S - 1; s >= 0 && e == hipSuccess && !pst; --s) {
      if (s + 2 < S) {  // set s & 1 is free once the reverse sweep of segment s + 2 has run
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&] { return stop || rev_done <= s + 2; });
        if (stop) break;
        lk.unlock();
        e = hipStreamWaitEvent(R, E(s + 2, 3), 0);
        if (e != hipSuccess) break;
      }
      e = hipEventRecord(E(s, 0), R);
      if (e == hipSuccess) pst = adj_recompute(c, s, R);
      if (e == hipSuccess && !pst) e = hipEventRecord(E(s, 1), R);
      std::lock_guard<std::mutex> lk(mu);
      if (e == hipSuccess && !pst) rec_done = s;
      cv.notify_all();
    }
    std::lock_guard<std::mutex> lk(mu);
    if (e != hipSuccess) {
      pst = ELBM_EDEVICE;
      perr = std::string("adjoint recomputation: ") + hipGetErrorString(e);
    } else if (pst) {
      perr = c->err;
    }
    if (pst) stop = true;
    cv.notify_all();
  });
  elbm_status st = ELBM_OK;
  hipError_t e = hipSuccess;
  for (int s = S - 1; s >= 0 && !st && e == hipSuccess; --s) {
    {
      std::unique_lock<std::mutex> lk(mu);
      cv.wait(lk, [&] { return stop || rec_done <= s; });
      if (stop) break;
    }
    e = hipStreamWaitEvent(c->stream, E(s, 1), 0);
    if (e == hipSuccess) e = hipEventRecord(E(s, 2), c->stream);
    A.rset = s & 1;
    const int Ks = std::min(A.K, A.n - s * A.K);
    // the transpose of the last reversed tick (coarse step 1, tick 1 of segment s + 1)
    // with the collision adjoint of this segment's last tick, now recomputed
    if (s + 1 < S && e == hipSuccess) st = adj_boundary(c, 1, Ks, s & 1);
    for (int k = Ks; k >= 1 && !st && e == hipSuccess; --k)
      for (int t = T; t >= 1 && !st; --t) {
        if (s == S - 1 && k == Ks && t == T) st = adj_collide_first(c, k, t);
        if (!st) st = adj_couple_part(c, k, t);
        if (st) break;
        if (t > 1) st = adj_boundary(c, t, k, s & 1);
        else if (k > 1) st = adj_boundary(c, 1, k - 1, s & 1);
        else if (s == 0) st = adj_transpose_last(c, 1);
      }
    if (!st && e == hipSuccess) e = hipEventRecord(E(s, 3), c->stream);
    std::lock_guard<std::mutex> lk(mu);
    if (!st && e == hipSuccess) rev_done = s;
    cv.notify_all();
  }
  {
    std::lock_guard<std::mutex> lk(mu);
    if (st || e != hipSuccess) stop = true;
    cv.notify_all();
  }
  producer.join();
  if (!st && e == hipSuccess && !pst) e = hipEventRecord(e_end, c->stream);
  hipStreamSynchronize(R);
  hipError_t se = hipStreamSynchronize(c->stream);
  if (e == hipSuccess) e = se;
  float rec = 0, rev = 0, tot = 0;
  if (!st && !pst && e == hipSuccess) {
    for (int s = 0; s < S && e == hipSuccess; ++s) {
      float a = 0, b = 0;
      e = hipEventElapsedTime(&a, E(s, 0), E(s, 1));
      if (e == hipSuccess) e = hipEventElapsedTime(&b, E(s, 2), E(s, 3));
      rec += a;
      rev += b;
    }
    if (e == hipSuccess) e = hipEventElapsedTime(&tot, e_begin, e_end);
  }
  for (auto &x : ev) hipEventDestroy(x);
  if (st) return st;
  if (pst) FAIL(c, pst, "%s", perr.c_str());
  if (e != hipSuccess) FAIL(c, ELBM_EDEVICE, "adjoint backward: %s", hipGetErrorString(e));
  A.ms[1] = rec;
  A.ms[2] = rev;
  A.ms[3] = tot;
  A.pending = false;
  return ELBM_OK;
}

elbm_status elbm_adjoint_read(elbm_ctx *c, int level, double *lam_dev, double *dJdF_dev) {
  if (!c) return ELBM_EINVAL;
  elbm_status s = check_level(c, level);
  if (s) return s;
  auto &A = c->adj;
  if (!A.bound || A.pending || A.n == 0) FAIL(c, ELBM_ESTATE, "adjoint_read before adjoint_backward");
  const Level &L = c->lev[level];
  Dims box;
  for (int a = 0; a < 3; ++a) box.n[a] = L.bn[a];
  const size_t tot = (size_t)(L.bn[0] * L.bn[1] * L.bn[2]);
  if (lam_dev) LCK(c, launch_zero(lam_dev, tot * c->Q * 8, c->stream));
  if (dJdF_dev) LCK(c, launch_zero(dJdF_dev, tot * c->D * 8, c->stream));
  LCK(c, launch_adj_read(c->D, c->storage, A.ws + A.o_lam[level][A.cur[level]], A.ws + A.o_lF[level],
                         (const LevelStatic *)(c->ws + c->o_levstatic), level, L.nb,
                         (const int32_t *)(c->ws + L.o_borg), box, lam_dev, dJdF_dev, c->stream));
  return ELBM_OK;
}

elbm_status elbm_adjoint_velocity(elbm_ctx *c, int level, const double *rho, const double *u, const double *noise,
                                  double *out) {
  if (!c || !rho || !u || !out) return ELBM_EINVAL;
  elbm_status s = check_level(c, level);
  if (s) return s;
  auto &A = c->adj;
  if (!A.bound || A.pending || A.n == 0) FAIL(c, ELBM_ESTATE, "adjoint_velocity before adjoint_backward");
  const Level &L = c->lev[level];
  const size_t tot = (size_t)(L.bn[0] * L.bn[1] * L.bn[2]);
  const size_t nd = tot * (1 + 2 * c->D + (noise ? c->Q : 0));
  double *d = nullptr;
  HIPCK(c, hipMalloc((void **)&d, nd * sizeof(double)));
  double *dr = d, *du = d + tot, *dout = d + tot * (1 + c->D), *dn = noise ? d + tot * (1 + 2 * c->D) : nullptr;
  hipError_t e = hipMemcpy(dr, rho, tot * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(du, u, tot * c->D * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess && noise) e = hipMemcpy(dn, noise, tot * c->Q * 8, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    hipFree(d);
    FAIL(c, ELBM_EDEVICE, "upload: %s", hipGetErrorString(e));
  }
  Dims box;
  for (int a = 0; a < 3; ++a) box.n[a] = L.bn[a];
  int rc = launch_zero(dout, tot * c->D * 8, c->stream);
  if (!rc)
    rc = launch_adj_velocity(c->D, c->storage, A.ws + A.o_lam[level][A.cur[level]],
                             (const LevelStatic *)(c->ws + c->o_levstatic), level, L.nb,
                             (const int32_t *)(c->ws + L.o_borg), box, dr, du, dn, dout, c->stream);
  if (!rc) rc = (int)hipStreamSynchronize(c->stream);
  if (!rc) rc = (int)hipMemcpy(out, dout, tot * c->D * 8, hipMemcpyDeviceToHost);
  hipFree(d);
  if (rc) FAIL(c, ELBM_EDEVICE, "adjoint_velocity: %s", hipGetErrorString((hipError_t)rc));
  return ELBM_OK;
}

elbm_status elbm_adjoint_timing(const elbm_ctx *c, double ms[4]) {
  if (!c || !ms) return ELBM_EINVAL;
  for (int q = 0; q < 4; ++q) ms[q] = c->adj.ms[q];
  return ELBM_OK;
}

}  // extern "C"
