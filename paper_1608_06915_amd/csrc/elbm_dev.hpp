// elbm_dev.hpp -- data layout shared by the host runtime and the HIP kernels.
//
// Storage: each level's nodes live in bricks of 16x4x4 (3-D) or 16x16 (2-D) nodes,
// allocated only where the level has nodes.  Populations are SoA inside a brick:
// pop[brick][i][node], node = x + BX*(y + BY*z), so a wavefront reads 64 consecutive
// nodes of one population.  Streaming pulls across brick faces through a 27-entry
// neighbour table per brick (periodic wrap folded into the table).
#pragma once
#include <stdint.h>

namespace elbm {

constexpr int MAXL = 8;
constexpr int BN = 256;  // nodes per brick (both dimensions)

template <int D> struct Brick;
template <> struct Brick<2> {
  static constexpr int BX = 16, BY = 16, BZ = 1, LX = 4, LY = 4;
};
template <> struct Brick<3> {
  static constexpr int BX = 16, BY = 4, BZ = 4, LX = 4, LY = 2;
};

// node class byte
enum : uint8_t {
  CLS_MODE = 0x3,      // 0: not stream-collided, 1: first substep only (inner layer), 2: every step
  CLS_LINKS = 0x4,     // mask holds bounce-back populations
  CLS_INLET = 0x8,     // mask holds populations entering through the inlet face
  CLS_OUTFLOW = 0x10,  // mask holds populations entering through the outflow face
  CLS_DRAG = 0x20,     // has links to solid nodes (momentum exchange)
  CLS_FLUID = 0x40,    // node exists and is not solid
};

enum { ST_F64 = 0, ST_F32 = 1, ST_F16S = 2, ST_BF16S = 3 };

struct WorkItem {  // one brick of one level in a stream-collide launch
  int32_t brick;
  uint8_t level;
  uint8_t thr;    // process nodes with mode >= thr
  uint8_t drag;   // brick holds drag nodes
  uint8_t flags;  // WI_PLAIN: every node is fluid, has mode >= thr and only plain links;
                  // WI_LINKS: some node has bounce-back, inlet or outflow links
};
enum : uint8_t { WI_PLAIN = 1, WI_LINKS = 2 };
static_assert(sizeof(WorkItem) == 8, "kernels read a WorkItem as one little-endian 64-bit word");

struct ItemRec {  // stream-collide work item with its 27 neighbour bricks (one scalar fetch)
  WorkItem w;
  int32_t nbr[27];  // neighbour brick per displacement code, -1 if absent
  int32_t pad[3];
};
static_assert(sizeof(ItemRec) == 128, "ItemRec layout");

struct GPoint {  // coarse-aligned interpolation point of an interface (gather phase)
  int32_t brick;
  uint16_t node;
  uint8_t level;  // level the value is read from
  uint8_t pair;   // interface pair index (parent level)
  int32_t slot;   // column in the staging buffer
};

struct CItem {  // node rebuilt by the coupling phase
  int32_t brick;
  uint16_t node;
  uint8_t level;  // level of the node written
  uint8_t kind;   // 0: fine interface node from stencil, 1: coarse ring node from fine twin
  int32_t a;      // kind 0: first stencil entry; kind 1: fine brick
  int32_t b;      // kind 0: stencil entries;     kind 1: fine node
};

struct StencilEntry {
  int32_t slot;  // staged row (untiled) or row in the tile's LDS copy (tiled)
  float w;
};

struct CTile {  // fine interface nodes of one brick whose stencils share staged rows
  int32_t item0, nitem;  // fine interface items
  int32_t pt0, npt;      // staged rows copied to LDS
  int32_t e0, ne;        // the items' stencil entries (contiguous), copied to LDS
};

struct LevelStatic {  // device-resident per-level constants and table pointers
  const uint8_t *cls;
  const uint32_t *mask;
  const int32_t *nbr;
  const float *weight;
  const float *force;  // [brick][D][BN], level-0 units, or null
  float *gamma;        // [brick][BN] or null
  double *drag;        // [brick][3]
  double beta;
  double F[3];   // uniform force density, level units
  double fscale; // 2^-l
  double hin[27];  // inlet populations minus weights
  int32_t oshift[3];
  int32_t nbricks;
};

struct PairStatic {
  double fac_pc;  // parent non-equilibrium to child scale: beta_c / (2 beta_f)
  double fac_cp;  // child non-equilibrium to parent scale: 2 beta_f / beta_c
  int32_t parent;
  int32_t pad;
};

// launch flags of the forward kernels
enum { FL_DRAG = 1, FL_GAMMA = 2 };

struct SCArgs {
  const ItemRec *items;
  int32_t n_items;
  int32_t remap;  // XCD-aware item mapping (0 identity, 1 by perm, B >= 2 runs of B items)
  int32_t flags;  // FL_DRAG: accumulate momentum exchange, FL_GAMMA: write gamma
  int32_t pad;
  const LevelStatic *lev;
  void *src[MAXL];
  void *dst[MAXL];
  const int32_t *perm;  // item of dispatch position q (remap 1), else null
};

struct GatherArgs {
  const GPoint *pts;
  int32_t n;
  int32_t stride;  // staging buffer column count
  void *stage;     // [1+D+Q][stride] compute type
  const LevelStatic *lev;
  const PairStatic *pairs;
  void *src[MAXL];
  const int32_t *nbr[MAXL];  // per level: the neighbour-brick table (as LevelStatic::nbr)
};

struct CoupleArgs {
  const CTile *tiles;     // fine interface tiles of the tick
  int32_t n_tiles;
  int32_t lds_rows;       // rows of the dynamic LDS buffer
  int32_t lds_ents;       // stencil entries of the dynamic LDS buffer (after the rows)
  const int32_t *tile_rows;  // staged row index per tile row
  const CItem *items;     // fine interface items (kind 0) referenced by the tiles
  const CItem *ring;      // coarse ring items (kind 1) of the tick
  int32_t n_ring;
  int32_t stride;
  const StencilEntry *sten;
  const void *stage;
  const LevelStatic *lev;
  const PairStatic *pairs;
  void *src[MAXL];
  void *dst[MAXL];
  int32_t flags;      // FL_GAMMA: write gamma
  int32_t lds_items;  // most fine interface nodes in one tile (the row area also holds their sums)
};

// ---------------------------------------------------------------- discrete adjoint
// Buffers of the reverse sweep, per level, in the compute type T (float, or double
// for FP64 storage), brick layout as the populations:
//   lam  adjoint of a post-collision state            [brick][Q][BN]
//   lg   adjoint of the post-stream state of a tick    [brick+1][Q][BN], the extra
//        brick stays zero and stands in for missing neighbours
//   lF   gradient wrt the per-node force field         [brick][D][BN]
struct AdjLevel {
  const uint32_t *amask;  // [brick][BN]: populations that an outflow node downstream copies
  int32_t zero_brick;     // index of the zero brick of lg
  int32_t pad;
};

struct AdjArgs {  // collision adjoint and streaming transpose over whole bricks
  const WorkItem *items;  // every brick of the arriving levels, thr of the tick
  int32_t n_items;
  int32_t drag_level;   // level whose momentum exchange is differentiated, or -1
  double drag_seed[3];  // direction / number of substeps of the average
  const LevelStatic *lev;
  const AdjLevel *alev;
  void *src[MAXL];  // forward state the tick read (storage type)
  void *lam[MAXL];  // adjoint of the tick's output (collision) / of its input (transpose)
  void *lg[MAXL];
  void *lF[MAXL];
};

struct AdjTCArgs {  // streaming transpose of one tick fused with the collision adjoint of the tick before
  const WorkItem *items;  // every brick of the levels of either tick; thr of the colliding tick
  int32_t n_items;
  int32_t drag_level;
  double drag_seed[3];
  const LevelStatic *lev;
  const AdjLevel *alev;
  void *src[MAXL];    // forward state the colliding tick read (storage type)
  void *lgsrc[MAXL];  // lg to transpose
  void *lam[MAXL];    // written by the transpose (tpose levels), else read by the collision
  void *lgdst[MAXL];  // lg written by the collision adjoint
  void *lF[MAXL];
  uint32_t tpose_mask, coll_mask;  // bit l: level l transposed / collided
};

struct AdjCoupleArgs {
  CoupleArgs c;     // tiles, items, ring, stencils, recomputed staged rows, src
  void *lam[MAXL];
  void *lg[MAXL];
  void *lF[MAXL];
  void *astage;     // [fine item][stage width]: adjoint of (rho~ - 1, u~, n~)
};

struct AdjPointArgs {
  const GPoint *pts;
  int32_t n;
  int32_t pad;
  const int32_t *tofs;            // per staged row: first transposed stencil entry (+1 sentinel)
  const StencilEntry *tsten;      // slot = fine item, w = weight
  const void *astage;
  const LevelStatic *lev;
  const PairStatic *pairs;
  void *src[MAXL];
  void *lg[MAXL];
};

struct AdjKEArgs {  // final kinetic energy: value, seed of lam, force-field seed
  const WorkItem *items;  // every brick of every level
  int32_t n_items;
  int32_t pad;
  const LevelStatic *lev;
  void *pop[MAXL];
  void *lam[MAXL];
  void *lF[MAXL];
  double *partials;  // [item][5], first entry used
};

// host-side launchers (kernels.hip)
struct LaunchCfg {
  int grid;
  int threads;
  int occ;   // stream-collide register-budget variant: 1 uncapped, 4 capped at 128 VGPRs
  int pipe;  // 1: persistent software-pipelined stream-collide (grid = wg_per_cu x CUs)
  // timing events (hipEvent_t) stamped with the kernel's own start and end by the
  // dispatch packet (hipExtLaunchKernel), or null
  void *ev0 = nullptr, *ev1 = nullptr;
};
int launch_stream_collide(int D, int st, const SCArgs &a, LaunchCfg cfg, void *stream);
int launch_gather(int D, int st, const GatherArgs &a, void *stream);
int launch_couple(int D, int st, const CoupleArgs &a, void *stream);
struct Dims {
  int64_t n[3];
};
int launch_init(int D, int st, void *pop, const LevelStatic *lev_dev, int level, int nbricks, const int32_t *borg,
                Dims box, const double *rho, const double *u, const double *noise, void *stream);
int launch_read(int D, int st, const void *pop, const LevelStatic *lev_dev, int level, int nbricks,
                const int32_t *borg, Dims box, double *rho, double *u, double *gamma, double *f, void *stream);
int launch_fill_nan(double *p, size_t count, void *stream);
int launch_stream_copy(void *dst, const void *src, size_t bytes, int grid, void *stream);
int launch_sample(int D, int st, const void *pop, const LevelStatic *lev_dev, int level, int n,
                  const int32_t *bricks, const int32_t *nodes, double *out, void *stream);
int launch_reduce(int D, int st, void *const *pops, const LevelStatic *lev_dev, const WorkItem *items, int n_items,
                  double *partials, double *result, void *stream);
int launch_force_scatter(int D, float *force, const double *F, int nbricks, const int32_t *borg, Dims box,
                         void *stream);
int stage_row_width(int D);
int couple_lds_stride(int D, int st);
int couple_max_rows(int D, int st);
int couple_max_entries();
int launch_zero(void *p, size_t bytes, void *stream);
int launch_adj_collide(int D, int st, const AdjArgs &a, void *stream);
int launch_adj_couple(int D, int st, const AdjCoupleArgs &a, void *stream);
int launch_adj_points(int D, int st, const AdjPointArgs &a, void *stream);
int launch_adj_tc(int D, int st, const AdjTCArgs &a, void *stream);
int launch_adj_transpose(int D, int st, const AdjArgs &a, void *stream);
int launch_adj_ke(int D, int st, const AdjKEArgs &a, double *result, void *stream);
int launch_adj_read(int D, int st, const void *lam, const void *lF, const LevelStatic *lev_dev, int level,
                    int nbricks, const int32_t *borg, Dims box, double *lam_out, double *lF_out, void *stream);
int launch_adj_velocity(int D, int st, const void *lam, const LevelStatic *lev_dev, int level, int nbricks,
                        const int32_t *borg, Dims box, const double *rho, const double *u, const double *noise,
                        double *out, void *stream);
int launch_copy(void *dst, const void *src, size_t bytes, void *stream);

}  // namespace elbm
