// kernels.hip -- gfx950 kernels of the refined KBC lattice Boltzmann path.
//
// All collision arithmetic works on shifted populations h_i = f_i - W_i, with
// rho = 1 + sum h and j = sum c h, which keeps FP32 rounding relative to the small
// deviations instead of to f itself.  The equilibrium of Eq. feq_iso is evaluated in
// an equivalent division-free per-axis form: with s = sqrt(1 + 3u^2) and
// sig = s - 1 = 3u^2 / (1 + s),
//   (2 - s) ((2u + s)/(1 - u))^c = 1 - sig        (c = 0)
//                                = 1 + 3cu + 2 sig (c = +-1),
// (multiply out (2-s)(2u+s) - (1-u) = (1-u)(3u + 2 sig)), so f_i^eq = rho W_i prod_a phi_a
// and f_i^eq - W_i = W_i q_i with q_i = (1 + drho) prod_a (1 + a_a) - 1 accumulated as
// q <- q + a + q a.  The inverse equilibrium for the entropic scalar product is the
// product of per-axis reciprocals (3 per axis instead of one per population).
#include "lbm_device.hpp"

#include <hip/hip_ext.h>

namespace elbm {

// ---------------------------------------------------------------- stream-collide
// OCC: minimum waves per SIMD requested from the register allocator (1: no cap,
// 4: at most 128 VGPRs); both variants are built and the launch configuration picks one.
// TWO: plain bricks take two nodes per thread (launched with BN/2 threads); built
// apart from the one-node kernel, whose register count it would otherwise set.
// PLAIN: every item is a plain brick (the caller launches the plain prefix of a tick's
// items with it); no code for walls, boundaries or drag, hence fewer registers.
template <int D, int ST, int OCC, bool TWO, bool PLAIN = false>
__global__ __launch_bounds__(256, OCC) void k_stream_collide(SCArgs a) {
  using C = Codec<ST>;
  using S = typename C::S;
  using T = typename C::T;
  constexpr int Q = nq<D>();
  __shared__ double s_red[3][8];
  const int G = gridDim.x;
  const int me = xcd_item(blockIdx.x, G, a.remap);
  for (int base = 0; base < a.n_items; base += G) {
    const int q = base + me;
    if (q >= a.n_items) break;
    const int idx = a.perm ? cst(a.perm)[q] : q;
    // the item, its level's constants and its neighbour bricks are wave-uniform:
    // scalar loads, issued together, with no dependent vector round trip
    cptr<ItemRec> rec = cst(a.items) + idx;
    const uint64_t wi = *(cptr<uint64_t>)rec;  // the WorkItem as one 8-byte word
    WorkItem w;
    w.brick = (int32_t)(uint32_t)wi;
    const int wl = (int)((wi >> 32) & 0xff), wthr = (int)((wi >> 40) & 0xff), wdrag = (int)((wi >> 48) & 0xff);
    const bool plain = PLAIN || ((wi >> 56) & WI_PLAIN) != 0;
    const bool links = !PLAIN && ((wi >> 56) & WI_LINKS) != 0;
    cptr<LevelStatic> Lc = cst(a.lev) + wl;
    cptr<int32_t> nbp = rec->nbr;
    const uint8_t *__restrict__ cls_p = Lc->cls + (size_t)w.brick * BN;
    const float *__restrict__ force_p = Lc->force;
    float *__restrict__ gamma_p = (a.flags & FL_GAMMA) ? Lc->gamma : nullptr;
    const T Fu[3] = {T(Lc->F[0]), T(Lc->F[1]), T(Lc->F[2])};
    const T fsc = T(Lc->fscale);
    const char *__restrict__ srcb = (const char *)a.src[wl];
    const uint32_t lbytes = (uint32_t)Lc->nbricks * brick_bytes<D, ST>();
    const Rsrc rsrc = buf_rsrc(a.src[wl], lbytes), rdst = buf_rsrc(a.dst[wl], lbytes);
    const uint32_t dbrick = (uint32_t)w.brick * brick_bytes<D, ST>();
    const T beta = T(Lc->beta);
    double fd[3] = {0, 0, 0};
    __shared__ uint32_t s_nbo[27];  // neighbour-brick byte offsets for per-lane lookups
    if (!plain) {
      if (threadIdx.x < 27) {
        const int nb = nbp[threadIdx.x];
        s_nbo[threadIdx.x] = (uint32_t)(nb < 0 ? 0 : nb) * brick_bytes<D, ST>();
      }
      __syncthreads();
    }
    if (TWO && plain) {
      // plain brick, two nodes per thread: both nodes' loads are issued before either
      // collision, doubling the bytes in flight per wavefront
      const int n0 = threadIdx.x, n1 = n0 + BN / 2;
      int x0, y0, z0, x1, y1, z1;
      node_xyz<D>(n0, x0, y0, z0);
      node_xyz<D>(n1, x1, y1, z1);
      if (D == 3) {
        z0 = __builtin_amdgcn_readfirstlane(z0);
        z1 = __builtin_amdgcn_readfirstlane(z1);
      }
      uint32_t mid[9], side0[9], side1[9];
      bulk_offsets<D, ST>([&](int q) { return (int)nbp[q]; }, z0, mid, side0);
      bulk_offsets<D, ST>([&](int q) { return (int)nbp[q]; }, z1, mid, side1);
      T h0[Q], h1[Q];
      pull_bulk<D, ST>(rsrc, mid, side0, BulkLane<D>(x0, y0, z0), h0);
      pull_bulk<D, ST>(rsrc, mid, side1, BulkLane<D>(x1, y1, z1), h1);
      auto one = [&](T (&h)[Q], int n) {
        T F[3] = {Fu[0], Fu[1], Fu[2]};
        if (force_p) {
          const float *fp = force_p + (size_t)w.brick * D * BN + n;
#pragma unroll
          for (int c = 0; c < D; ++c) F[c] += T(fp[c * BN]) * fsc;
        }
        const bool hf = (F[0] != T(0)) || (F[1] != T(0)) || (F[2] != T(0));
        const T g = kbc_collide<D, T>(h, beta, F, hf, [&](int i, T v) {
          C::stb(rdst, (uint32_t)(n * (int)sizeof(S)), dbrick + (uint32_t)(i * BN * (int)sizeof(S)), v, T(wgt<D>(i)));
        });
        if (gamma_p) gamma_p[(size_t)w.brick * BN + n] = (float)g;
      };
      one(h0, n0);
      one(h1, n1);
      continue;
    }
    for (int n = threadIdx.x; n < BN; n += blockDim.x) {
      uint8_t cls = CLS_FLUID | 2;
      uint32_t lmask = 0;
      if (!plain) {
        // in a brick with special links the node's link mask is loaded beside its class
        // (not after it)
        cls = cls_p[n];
        if (links) lmask = Lc->mask[(size_t)w.brick * BN + n];
        if ((cls & CLS_MODE) < wthr) continue;
      }
      int x, y, z;
      node_xyz<D>(n, x, y, z);
      if (D == 3) z = __builtin_amdgcn_readfirstlane(z);  // one z-slice per wavefront
      T h[Q];
      uint32_t mask = 0;
      // a wavefront with any special lane pulls every lane through pull_links (plain
      // lanes have an empty mask there), so it runs one pull instead of two
      const bool special = !plain && (cls & (CLS_LINKS | CLS_INLET | CLS_OUTFLOW));
      if (!plain && __builtin_amdgcn_ballot_w64(special) != 0) {
        mask = special ? lmask : 0u;
        uint32_t mid[9], side[9];
        bulk_offsets<D, ST>([&](int q) { return (int)nbp[q]; }, z, mid, side);
        const BulkLane<D> bl(x, y, z);
        pull_links<D, ST>(rsrc, mid, side, bl, [&](int q) { return s_nbo[q]; }, dbrick, x, y, z, n, cls, mask, Lc, h);
      } else {
        uint32_t mid[9], side[9];
        bulk_offsets<D, ST>([&](int q) { return (int)nbp[q]; }, z, mid, side);
        const BulkLane<D> bl(x, y, z);
        pull_bulk<D, ST>(rsrc, mid, side, bl, h);
      }
      T F[3] = {Fu[0], Fu[1], Fu[2]};
      if (force_p) {
        const float *fp = force_p + (size_t)w.brick * D * BN + n;
#pragma unroll
        for (int c = 0; c < D; ++c) F[c] += T(fp[c * BN]) * fsc;
      }
      const bool hf = (F[0] != T(0)) || (F[1] != T(0)) || (F[2] != T(0));
      const T g = kbc_collide<D, T>(h, beta, F, hf, [&](int i, T v) {
        C::stb(rdst, (uint32_t)(n * (int)sizeof(S)), dbrick + (uint32_t)(i * BN * (int)sizeof(S)), v, T(wgt<D>(i)));
      });
      if (gamma_p) gamma_p[(size_t)w.brick * BN + n] = (float)g;
      if (!plain && (cls & CLS_DRAG) && (a.flags & FL_DRAG)) {
        // population i leaves towards x + c_i; that node is solid when population Q-1-i
        // bounced back: momentum exchange 2 c_i f'_i, from the values just stored (all
        // read back at once, then accumulated under the link mask)
        T r[Q];
        static_for<0, Q>([&](auto I) {
          constexpr int i = decltype(I)::value;
          r[i] = C::ldb(rdst, (uint32_t)(n * (int)sizeof(S)), dbrick + (uint32_t)(i * BN * (int)sizeof(S)),
                        T(wgt<D>(i)));
        });
        static_for<0, Q>([&](auto I) {
          constexpr int i = decltype(I)::value;
          if ((mask >> (Q - 1 - i)) & 1u) {
            const double fi = wgt<D>(i) + (double)r[i];
            fd[0] += 2.0 * (double)cxo(i) * fi;
            fd[1] += 2.0 * (double)cyo(i) * fi;
            fd[2] += 2.0 * (double)czo<D>(i) * fi;
          }
        });
      }
    }
    if (!plain) __syncthreads();  // s_nbo is rewritten by the next item
    if (wdrag && (a.flags & FL_DRAG)) {  // deterministic block reduction of the momentum exchange
      double v[3] = {fd[0], fd[1], fd[2]};
#pragma unroll
      for (int k = 0; k < 3; ++k)
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_down(v[k], off, 64);
      const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
      if (lane == 0)
        for (int k = 0; k < 3; ++k) s_red[k][wave] = v[k];
      __syncthreads();
      if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int k = 0; k < 3; ++k) {
          double s = 0;
          for (int q = 0; q < nw; ++q) s += s_red[k][q];
          Lc->drag[(size_t)w.brick * 3 + k] += s;
        }
      }
    }
  }
}

// ---------------------------------------------------------------- stream-collide, pipelined
// Persistent variant for plain bricks (every node fluid, updated, plain links only):
// workgroup g processes items g, g+G, g+2G, ...  The records of a chunk of its items
// are staged in LDS once; each thread (one node of the brick) issues the loads of its
// node in the next brick before it collides its node in the current brick (two
// register buffers of raw stored values, decoded only when used), so load latency
// overlaps the collision arithmetic.  Straight-line code: no per-node branches.
constexpr int PIPE_RECS = 16;

template <int D, int ST> __global__ __launch_bounds__(256, 2) void k_sc_pipe(SCArgs a) {
  using C = Codec<ST>;
  using S = typename C::S;
  using T = typename C::T;
  constexpr int Q = nq<D>();
  __shared__ ItemRec srec[PIPE_RECS];
  const int G = gridDim.x;
  const int me = xcd_item(blockIdx.x, G, a.remap);
  if (me >= a.n_items) return;
  const int cnt = (a.n_items - me + G - 1) / G;
  const int n = threadIdx.x;
  int x, y, z;
  node_xyz<D>(n, x, y, z);
  if (D == 3) z = __builtin_amdgcn_readfirstlane(z);  // one z-slice per wavefront
  const BulkLane<D> bl(x, y, z);
  auto level_of = [&](int j) { return __builtin_amdgcn_readfirstlane((int)srec[j].w.level); };
  auto brick_of = [&](int j) { return __builtin_amdgcn_readfirstlane((int)srec[j].w.brick); };
  // all loads of item j (populations and the node's force field) are issued together:
  // the memory counter completes in order, so a later load would wait for the prefetch
  auto fetch = [&](int j, S (&r)[Q], float (&rf)[3]) {
    const int l = level_of(j);
    cptr<LevelStatic> Lc = cst(a.lev) + l;
    const Rsrc rs = buf_rsrc(a.src[l], (uint32_t)Lc->nbricks * brick_bytes<D, ST>());
    uint32_t mid[9], side[9];
    bulk_offsets<D, ST>([&](int k) { return __builtin_amdgcn_readfirstlane(srec[j].nbr[k]); }, z, mid, side);
    pull_bulk_with<D, ST>(mid, side, bl, [&](int i, uint32_t v, uint32_t s) { r[i] = C::ldr(rs, v, s); });
    rf[0] = rf[1] = rf[2] = 0.f;
    const float *force_p = Lc->force;
    if (force_p) {
      const Rsrc rfc = buf_rsrc(force_p, (uint32_t)Lc->nbricks * D * BN * 4u);
      const uint32_t fb = (uint32_t)brick_of(j) * (uint32_t)(D * BN * 4);
#pragma unroll
      for (int c = 0; c < D; ++c)
        rf[c] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rfc, (uint32_t)(n * 4),
                                                                               fb + (uint32_t)(c * BN * 4), 0));
    }
  };
  auto finish = [&](int j, const S (&r)[Q], const float (&rf)[3]) {
    const int l = level_of(j), brick = brick_of(j);
    cptr<LevelStatic> Lc = cst(a.lev) + l;
    T h[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) h[i] = C::dec(r[i], T(wgt<D>(i)));
    const uint32_t dbrick = (uint32_t)brick * brick_bytes<D, ST>();
    const Rsrc rd = buf_rsrc(a.dst[l], (uint32_t)Lc->nbricks * brick_bytes<D, ST>());
    T F[3] = {T(Lc->F[0]), T(Lc->F[1]), T(Lc->F[2])};
    if (Lc->force) {
#pragma unroll
      for (int c = 0; c < D; ++c) F[c] += T(rf[c]) * T(Lc->fscale);
    }
    const bool hf = (F[0] != T(0)) || (F[1] != T(0)) || (F[2] != T(0));
    const T g = kbc_collide<D, T>(h, T(Lc->beta), F, hf, [&](int i, T v) {
      C::stb(rd, (uint32_t)(n * (int)sizeof(S)), dbrick + (uint32_t)(i * BN * (int)sizeof(S)), v, T(wgt<D>(i)));
    });
    if ((a.flags & FL_GAMMA) && Lc->gamma) Lc->gamma[(size_t)brick * BN + n] = (float)g;
  };
  for (int c0 = 0; c0 < cnt; c0 += PIPE_RECS) {
    const int m = cnt - c0 < PIPE_RECS ? cnt - c0 : PIPE_RECS;
    for (int t = threadIdx.x; t < m * 32; t += blockDim.x) {
      const int r = t >> 5, q = t & 31;
      const int pos = me + (c0 + r) * G;
      const int idx = a.perm ? a.perm[pos] : pos;
      ((uint32_t *)srec)[t] = ((const uint32_t *)(a.items + idx))[q];
    }
    __syncthreads();
    S hA[Q], hB[Q];
    float fA[3], fB[3];
    fetch(0, hA, fA);
    for (int j = 0; j < m; j += 2) {
      if (j + 1 < m) fetch(j + 1, hB, fB);
      finish(j, hA, fA);
      if (j + 1 >= m) break;
      if (j + 2 < m) fetch(j + 2, hA, fA);
      finish(j + 1, hB, fB);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- interface gather
// Post-stream (rho - 1, u, f^neq) at coarse-aligned interpolation points, parent
// values brought to child scale (Eq. f_neq_rescaling_iso); one staged row per point.

template <int D, int ST> __global__ __launch_bounds__(256) void k_gather(GatherArgs a) {
  using C = Codec<ST>;
  using T = typename C::T;
  constexpr int Q = nq<D>();
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.n) return;
  const GPoint g = a.pts[p];
  // the level's population buffer and neighbour table chosen among kernel arguments
  // (selects, not a memory round trip on the lane's level)
  // (the empty asm keeps each argument in scalar registers, so that the choice stays a
  // select and is not turned back into an indexed load from the argument segment)
  const char *srcb = nullptr;
  const int32_t *nbt = nullptr;
#pragma unroll
  for (int l = 0; l < MAXL; ++l) {
    const char *sl = (const char *)a.src[l];
    const int32_t *nl = a.nbr[l];
    asm volatile("" : "+s"(sl), "+s"(nl));
    if (g.level == l) {
      srcb = sl;
      nbt = nl;
    }
  }
  const int32_t *nb = nbt + (size_t)g.brick * 27;
  auto boff = [&](int code) { return (uint32_t)nb[code] * brick_bytes<D, ST>(); };
  int x, y, z;
  node_xyz<D>(g.node, x, y, z);
  const Lane<D> ln(x, y, z);
  T h[Q];
  pull_plain<D, ST>(srcb, boff, ln, h);
  T drho, j[3];
  moments<D, T>(h, drho, j);
  const T ir = rcp(T(1) + drho);
  T u[3] = {j[0] * ir, j[1] * ir, j[2] * ir};
  T q[Q];
  eq_dev<D, T>(drho, u, q);
  const PairStatic &P = a.pairs[g.pair];
  const T fac = (g.level == P.parent) ? T(P.fac_pc) : T(1);
  T *row = (T *)a.stage + (size_t)g.slot * stage_width<D>();
  row[0] = drho;
#pragma unroll
  for (int c = 0; c < D; ++c) row[1 + c] = u[c];
#pragma unroll
  for (int i = 0; i < Q; ++i) row[1 + D + i] = fac * (h[i] - T(wgt<D>(i)) * q[i]);
  if (D == 3) row[31] = T(0);
}

// ---------------------------------------------------------------- interface coupling
// Fine interface nodes: tensor four-point reconstruction (Eq. interp) of rho, u and
// f^neq from staged rows, f = f^eq(rho~, u~) + f~neq; coarse ring nodes: co-located
// fine post-stream state with f^neq brought to coarse scale.  Both then collide with
// their own level's parameters (Sec. III.C steps 3-5).
// Fine interface nodes are processed per tile (one workgroup per fine brick): the
// staged rows its stencils use are copied to LDS once; then every (node, 4-value
// column) pair is one lane's task, accumulating that column over the node's stencil
// (the lanes of a node share its entry count, so a wavefront runs no idle
// iterations); the sums go back to LDS over the rows and one lane per node collides.
// Ring nodes are handled by the leading workgroups.
constexpr int COUPLE_LDS_BYTES = 48 * 1024;
constexpr int COUPLE_THREADS = 256;
static_assert(BN <= COUPLE_THREADS, "the collision phase of a tile takes one node per thread");
template <int D, typename T> __host__ __device__ constexpr int couple_rows() {
  return COUPLE_LDS_BYTES / (lds_stride<D, T>() * (int)sizeof(T));
}

template <int D, int ST> __device__ inline void couple_finish(const CoupleArgs &a, const CItem &c,
                                                             typename Codec<ST>::T (&h)[nq<D>()]) {
  using C = Codec<ST>;
  using S = typename C::S;
  using T = typename C::T;
  constexpr int Q = nq<D>();
  const LevelStatic &L = a.lev[c.level];
  T F[3];
  node_force<D, T>(L, c.brick, c.node, F);
  const bool hf = (F[0] != T(0)) || (F[1] != T(0)) || (F[2] != T(0));
  S *o = (S *)a.dst[c.level] + (size_t)c.brick * Q * BN + c.node;
  const T g = kbc_collide<D, T>(h, T(L.beta), F, hf, [&](int i, T v) { C::st(o + i * BN, v, T(wgt<D>(i))); });
  if (L.gamma && (a.flags & FL_GAMMA)) L.gamma[(size_t)c.brick * BN + c.node] = (float)g;
}

// the same for a node of a tile: the level is uniform over the workgroup, so its
// constants are scalar loads
template <int D, int ST> __device__ inline void couple_finish_u(const CoupleArgs &a, cptr<LevelStatic> Lc, int lvl,
                                                               const CItem &c, typename Codec<ST>::T (&h)[nq<D>()]) {
  using C = Codec<ST>;
  using S = typename C::S;
  using T = typename C::T;
  constexpr int Q = nq<D>();
  T F[3] = {T(Lc->F[0]), T(Lc->F[1]), T(Lc->F[2])};
  const float *force = Lc->force;
  if (force) {
    const float *fp = force + (size_t)c.brick * D * BN + c.node;
#pragma unroll
    for (int k = 0; k < D; ++k) F[k] += T(fp[k * BN]) * T(Lc->fscale);
  }
  const bool hf = (F[0] != T(0)) || (F[1] != T(0)) || (F[2] != T(0));
  S *o = (S *)a.dst[lvl] + (size_t)c.brick * Q * BN + c.node;
  const T g = kbc_collide<D, T>(h, T(Lc->beta), F, hf, [&](int i, T v) { C::st(o + i * BN, v, T(wgt<D>(i))); });
  float *gam = Lc->gamma;
  if (gam && (a.flags & FL_GAMMA)) gam[(size_t)c.brick * BN + c.node] = (float)g;
}

template <int D, int ST> __global__ __launch_bounds__(COUPLE_THREADS, ST == ST_F64 ? 2 : 4) void k_couple(CoupleArgs a) {
  using C = Codec<ST>;
  using T = typename C::T;
  using V = typename V4<T>::type;
  constexpr int Q = nq<D>();
  constexpr int SW = stage_width<D>();
  constexpr int NV = SW / 4;  // 4-element columns of a staged row
  constexpr int SL = lds_stride<D, T>();
  constexpr int NT = COUPLE_THREADS;
  constexpr int TPT = (BN * NV + NT - 1) / NT;  // column tasks per lane (a tile holds at most BN nodes)
  extern __shared__ __align__(16) unsigned char couple_lds[];
  T *rows = (T *)couple_lds;
  // ring workgroups first: each is one long dependent chain (27 pulls, then the
  // collision) and would otherwise form the tail of the launch
  const int ring_blocks = (a.n_ring + NT - 1) / NT;
  const int tb = (int)blockIdx.x - ring_blocks;
  if (tb >= 0) {
    const CTile t = a.tiles[tb];
    const V *stage = (const V *)a.stage;
    // entries packed to 4 bytes: tile-local row (16 bits) and the weight in FP16 (the
    // weights are products of -1/16, 9/16 and 1: exact in FP16); the row area also
    // holds the per-node sums of the last phase
    const int rcap = a.lds_rows > a.lds_items ? a.lds_rows : a.lds_items;
    uint32_t *ents = (uint32_t *)(rows + (size_t)rcap * SL);
    const int tid = (int)threadIdx.x;
    const int ntask = t.nitem * NV, nrow = t.npt * NV;
    // every global load of the tile is issued before the first barrier, none waiting on
    // another but the staged rows on their indices: the record of the node this lane
    // collides, the stencil ranges of its column tasks, the row indices and entries
    // (the loads are unconditional, with indices clamped into the tile -- a tile has at
    // least one node, row and entry -- so that they are issued back to back; a load
    // under its own condition is waited for inside that condition)
    const CItem cn = a.items[t.item0 + (tid < t.nitem ? tid : 0)];
    int ea[TPT], eb[TPT];
#pragma unroll
    for (int p = 0; p < TPT; ++p) {
      const int k = p * NT + tid;
      const CItem c = a.items[t.item0 + (k < ntask ? k : 0) / NV];
      ea[p] = c.a;
      eb[p] = c.b;
    }
#pragma unroll
    for (int p = 0; p < TPT; ++p) {
      const bool in = p * NT + tid < ntask;
      ea[p] = in ? ea[p] - t.e0 : 0;
      eb[p] = in ? eb[p] : 0;
    }
    constexpr int RC = 8;  // row columns and entries per lane per round
    for (int k0 = 0; k0 < nrow || k0 < t.ne; k0 += RC * NT) {
      int ri[RC];
      StencilEntry se[RC];
#pragma unroll
      for (int j = 0; j < RC; ++j) {
        const int k = k0 + j * NT + tid;
        ri[j] = a.tile_rows[t.pt0 + (k < nrow ? k : 0) / NV];
        se[j] = a.sten[t.e0 + (k < t.ne ? k : 0)];
      }
      V rv[RC];
#pragma unroll
      for (int j = 0; j < RC; ++j) {
        const int k = k0 + j * NT + tid;
        rv[j] = stage[(size_t)ri[j] * NV + (k < nrow ? k : 0) % NV];
      }
#pragma unroll
      for (int j = 0; j < RC; ++j) {
        const int k = k0 + j * NT + tid;
        if (k < nrow) ((V *)rows)[(k / NV) * (SL / 4) + k % NV] = rv[j];
        if (k < t.ne) ents[k] = (uint32_t)se[j].slot | ((uint32_t)__half_as_ushort(__float2half_rn(se[j].w)) << 16);
      }
    }
    __syncthreads();
    T ax[TPT], ay[TPT], az[TPT], aw[TPT];
#pragma unroll
    for (int p = 0; p < TPT; ++p) {
      ax[p] = ay[p] = az[p] = aw[p] = T(0);
      const int k = p * NT + tid;
      if (k < ntask) {
        const int col = k % NV;
        auto acc1 = [&](uint32_t s, const V &r) {
          const T w = T(__half2float(__ushort_as_half((uint16_t)(s >> 16))));
          ax[p] = fma(w, r.x, ax[p]);
          ay[p] = fma(w, r.y, ay[p]);
          az[p] = fma(w, r.z, az[p]);
          aw[p] = fma(w, r.w, aw[p]);
        };
        auto row = [&](uint32_t s) { return ((const V *)(rows + (s & 0xffffu) * SL))[col]; };
        int e = ea[p];
        const int e1 = ea[p] + eb[p];
        // four entries, then their four rows, in flight at once; summed in entry order
        for (; e + 4 <= e1; e += 4) {
          const uint32_t s0 = ents[e], s1 = ents[e + 1], s2 = ents[e + 2], s3 = ents[e + 3];
          const V r0 = row(s0), r1 = row(s1), r2 = row(s2), r3 = row(s3);
          acc1(s0, r0);
          acc1(s1, r1);
          acc1(s2, r2);
          acc1(s3, r3);
        }
        for (; e < e1; ++e) {
          const uint32_t s0 = ents[e];
          acc1(s0, row(s0));
        }
      }
    }
    __syncthreads();  // the staged rows are no longer read
#pragma unroll
    for (int p = 0; p < TPT; ++p) {
      const int k = p * NT + (int)threadIdx.x;
      if (k < ntask) {
        const int node = k / NV, col = k - node * NV;
        V v;
        v.x = ax[p];
        v.y = ay[p];
        v.z = az[p];
        v.w = aw[p];
        ((V *)rows)[node * (SL / 4) + col] = v;
      }
    }
    __syncthreads();
    if (tid < t.nitem) {  // a tile holds at most BN = NT nodes
      const int lvl = __builtin_amdgcn_readfirstlane((int)cn.level);
      T acc[SW];
      const V *row = (const V *)(rows + tid * SL);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const V r = row[v];
        acc[4 * v + 0] = r.x;
        acc[4 * v + 1] = r.y;
        acc[4 * v + 2] = r.z;
        acc[4 * v + 3] = r.w;
      }
      T u[3] = {acc[1], acc[2], D == 3 ? acc[3] : T(0)};
      T q[Q], h[Q];
      eq_dev<D, T>(acc[0], u, q);
#pragma unroll
      for (int i = 0; i < Q; ++i) h[i] = acc[1 + D + i] + T(wgt<D>(i)) * q[i];
      couple_finish_u<D, ST>(a, cst(a.lev) + lvl, lvl, cn, h);
    }
    return;
  }
  const int t = (int)blockIdx.x * NT + (int)threadIdx.x;
  if (t >= a.n_ring) return;
  const CItem c = a.ring[t];
  const int fl = c.level + 1;
  const LevelStatic &Lf = a.lev[fl];
  const char *srcb = (const char *)a.src[fl];
  const int32_t *nb = Lf.nbr + (size_t)c.a * 27;
  auto boff = [&](int code) { return (uint32_t)nb[code] * brick_bytes<D, ST>(); };
  int x, y, z;
  node_xyz<D>(c.b, x, y, z);
  const Lane<D> ln(x, y, z);
  T h[Q];
  pull_plain<D, ST>(srcb, boff, ln, h);
  T drho, j[3];
  moments<D, T>(h, drho, j);
  const T ir = rcp(T(1) + drho);
  T u[3] = {j[0] * ir, j[1] * ir, j[2] * ir};
  T q[Q];
  eq_dev<D, T>(drho, u, q);
  const T fac = T(a.pairs[c.level].fac_cp);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const T heq = T(wgt<D>(i)) * q[i];
    h[i] = heq + fac * (h[i] - heq);
  }
  couple_finish<D, ST>(a, c, h);
}

// ---------------------------------------------------------------- initialisation
template <int D, int ST>
__global__ __launch_bounds__(256) void k_init(typename Codec<ST>::S *pop, const LevelStatic *lev, int level,
                                              const int32_t *borg, Dims box, const double *rho, const double *u,
                                              const double *noise) {
  using C = Codec<ST>;
  using T = typename C::T;
  constexpr int Q = nq<D>();
  const int b = blockIdx.x, n = threadIdx.x;
  const LevelStatic &L = lev[level];
  const uint8_t cls = L.cls[(size_t)b * BN + n];
  typename C::S *o = pop + (size_t)b * Q * BN + n;
  if (!(cls & CLS_FLUID)) {
#pragma unroll
    for (int i = 0; i < Q; ++i) C::st(o + i * BN, T(0), T(wgt<D>(i)));
    return;
  }
  int x, y, z;
  node_xyz<D>(n, x, y, z);
  const int64_t X = borg[3 * b] + x, Y = borg[3 * b + 1] + y, Z = borg[3 * b + 2] + z;
  const int64_t tot = box.n[0] * box.n[1] * box.n[2];
  const int64_t k = X + box.n[0] * (Y + box.n[1] * Z);
  double uu[3] = {u[k], u[tot + k], D == 3 ? u[2 * tot + k] : 0.0};
  double q[Q];
  eq_dev<D, double>(rho[k] - 1.0, uu, q);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    double hi = wgt<D>(i) * q[i];
    if (noise) hi += wgt<D>(i) * (1.0 + q[i]) * noise[(int64_t)i * tot + k];
    C::st(o + i * BN, T(hi), T(wgt<D>(i)));
  }
}

// ---------------------------------------------------------------- readout
template <int D, int ST>
__global__ __launch_bounds__(256) void k_read(const typename Codec<ST>::S *pop, const LevelStatic *lev, int level,
                                              const int32_t *borg, Dims box, double *rho, double *u, double *gam,
                                              double *f) {
  using C = Codec<ST>;
  using T = typename C::T;
  constexpr int Q = nq<D>();
  const int b = blockIdx.x, n = threadIdx.x;
  const LevelStatic &L = lev[level];
  const uint8_t cls = L.cls[(size_t)b * BN + n];
  if (!(cls & CLS_FLUID)) return;
  int x, y, z;
  node_xyz<D>(n, x, y, z);
  const int64_t X = borg[3 * b] + x, Y = borg[3 * b + 1] + y, Z = borg[3 * b + 2] + z;
  if (X >= box.n[0] || Y >= box.n[1] || Z >= box.n[2]) return;
  const int64_t tot = box.n[0] * box.n[1] * box.n[2];
  const int64_t k = X + box.n[0] * (Y + box.n[1] * Z);
  const typename C::S *p = pop + (size_t)b * Q * BN + n;
  double r = 0, j[3] = {0, 0, 0};
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const double fi = wgt<D>(i) + (double)C::ld(p + i * BN, T(wgt<D>(i)));
    r += fi;
    j[0] += cxo(i) * fi;
    j[1] += cyo(i) * fi;
    j[2] += czo<D>(i) * fi;
    if (f) f[(int64_t)i * tot + k] = fi;
  }
  double F[3];
  node_force<D, double>(L, b, n, F);
  if (rho) rho[k] = r;
  if (u)
    for (int c = 0; c < D; ++c) u[(int64_t)c * tot + k] = j[c] / r - 0.5 * F[c] / r;
  if (gam) gam[k] = L.gamma ? (double)L.gamma[(size_t)b * BN + n] : 2.0;
}

// Plain streaming copy (16-byte loads, non-temporal 16-byte stores, grid-stride): the
// read + write bandwidth HBM sustains for a pure stream, the practical ceiling the
// stream-collide's traffic is compared against.
__global__ __launch_bounds__(256) void k_stream_copy(const float4 *__restrict__ src, float4 *__restrict__ dst,
                                                     size_t n) {
  typedef float v4 __attribute__((ext_vector_type(4)));
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t step = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += step) {
    const float4 v = src[i];
    const v4 w = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(w, (v4 *)&dst[i]);
  }
}

__global__ void k_fill_nan(double *p, size_t count) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t step = (size_t)gridDim.x * blockDim.x;
  for (; i < count; i += step) p[i] = __longlong_as_double(0x7ff8000000000000LL);
}

template <int D, int ST>
__global__ void k_sample(const typename Codec<ST>::S *pop, int n, const int32_t *bricks, const int32_t *nodes,
                         double *out) {
  using C = Codec<ST>;
  using T = typename C::T;
  constexpr int Q = nq<D>();
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int b = bricks[t], nd = nodes[t];
  for (int i = 0; i < Q; ++i) {
    double v = __longlong_as_double(0x7ff8000000000000LL);
    if (b >= 0) v = wgt<D>(i) + (double)C::ld(pop + ((size_t)b * Q + i) * BN + nd, T(wgt<D>(i)));
    out[(size_t)t * Q + i] = v;
  }
}

// ---------------------------------------------------------------- reductions
// Owned-volume mass deviation, momentum (mid-step) and unstable-node count per
// brick, reduced per workgroup in a fixed order, then summed in a fixed order by one
// workgroup: bitwise reproducible.
struct ReduceArgs {
  const WorkItem *items;
  int n_items;
  const LevelStatic *lev;
  void *pop[MAXL];
  double *partials;
};

template <int D, int ST> __global__ __launch_bounds__(256) void k_reduce(ReduceArgs a) {
  using C = Codec<ST>;
  using T = typename C::T;
  constexpr int Q = nq<D>();
  __shared__ double s[5][4];
  const int it = blockIdx.x;
  const WorkItem w = a.items[it];
  const LevelStatic &L = a.lev[w.level];
  const typename C::S *p = (const typename C::S *)a.pop[w.level] + (size_t)w.brick * Q * BN + threadIdx.x;
  const uint8_t cls = L.cls[(size_t)w.brick * BN + threadIdx.x];
  double v[5] = {0, 0, 0, 0, 0};
  if (cls & CLS_FLUID) {
    T drho = 0, j[3] = {0, 0, 0};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const T hi = C::ld(p + i * BN, T(wgt<D>(i)));
      drho += hi;
      j[0] += T(cxo(i)) * hi;
      j[1] += T(cyo(i)) * hi;
      j[2] += T(czo<D>(i)) * hi;
    }
    const double wt = (double)L.weight[(size_t)w.brick * BN + threadIdx.x];
    double F[3];
    node_force<D, double>(L, w.brick, threadIdx.x, F);
    v[0] = wt * (double)drho;
    for (int c = 0; c < 3; ++c) v[1 + c] = wt * ((double)j[c] - 0.5 * F[c]);
    const double r = 1.0 + (double)drho;
    bool bad = !(r > 0.0) || !isfinite(r);
    for (int c = 0; c < D; ++c) bad = bad || !(fabs((double)j[c] / r) < 1.0);
    v[4] = bad ? 1.0 : 0.0;
  }
  for (int k = 0; k < 5; ++k)
    for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_down(v[k], off, 64);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0)
    for (int k = 0; k < 5; ++k) s[k][wave] = v[k];
  __syncthreads();
  if (threadIdx.x < 5) {
    double t = 0;
    for (int q = 0; q < 4; ++q) t += s[threadIdx.x][q];
    a.partials[(size_t)it * 5 + threadIdx.x] = t;
  }
}

__global__ __launch_bounds__(256) void k_reduce_final(const double *partials, int n, double *out) {
  __shared__ double s[5][256];
  double v[5] = {0, 0, 0, 0, 0};
  for (int i = threadIdx.x; i < n; i += 256)
    for (int k = 0; k < 5; ++k) v[k] += partials[(size_t)i * 5 + k];
  for (int k = 0; k < 5; ++k) s[k][threadIdx.x] = v[k];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int k = 0; k < 5; ++k) s[k][threadIdx.x] += s[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 5) out[threadIdx.x] = s[threadIdx.x][0];
}

template <int D>
__global__ void k_force_scatter(float *force, const double *F, const int32_t *borg, Dims box) {
  const int b = blockIdx.x, n = threadIdx.x;
  int x, y, z;
  node_xyz<D>(n, x, y, z);
  const int64_t X = borg[3 * b] + x, Y = borg[3 * b + 1] + y, Z = borg[3 * b + 2] + z;
  float *o = force + (size_t)b * D * BN + n;
  if (X >= box.n[0] || Y >= box.n[1] || Z >= box.n[2]) {
    for (int c = 0; c < D; ++c) o[c * BN] = 0.f;
    return;
  }
  const int64_t tot = box.n[0] * box.n[1] * box.n[2];
  const int64_t k = X + box.n[0] * (Y + box.n[1] * Z);
  for (int c = 0; c < D; ++c) o[c * BN] = (float)F[(int64_t)c * tot + k];
}

__global__ void k_zero(uint32_t *p, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t step = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += step) p[i] = 0u;
}

// ---------------------------------------------------------------- launchers
static int ck() { return (int)hipGetLastError(); }

#define ELBM_DISPATCH(D, st, CALL)                            \
  do {                                                        \
    if (D == 2) {                                             \
      constexpr int DD = 2;                                   \
      switch (st) {                                           \
        case ST_F64: { constexpr int SS = ST_F64; CALL; } break;   \
        case ST_F32: { constexpr int SS = ST_F32; CALL; } break;   \
        case ST_F16S: { constexpr int SS = ST_F16S; CALL; } break; \
        default: { constexpr int SS = ST_BF16S; CALL; } break;     \
      }                                                       \
    } else {                                                  \
      constexpr int DD = 3;                                   \
      switch (st) {                                           \
        case ST_F64: { constexpr int SS = ST_F64; CALL; } break;   \
        case ST_F32: { constexpr int SS = ST_F32; CALL; } break;   \
        case ST_F16S: { constexpr int SS = ST_F16S; CALL; } break; \
        default: { constexpr int SS = ST_BF16S; CALL; } break;     \
      }                                                       \
    }                                                         \
  } while (0)

// One stream-collide launch; with timing events the dispatch packet stamps them with the
// kernel's start and end (no host-side marker packets around the kernel).
template <int D, int ST, int OCC, bool TWO, bool PLAIN>
static void go_sc(int grid, int thr, const SCArgs &a, const LaunchCfg &cfg, hipStream_t s) {
  if (cfg.ev0)
    hipExtLaunchKernelGGL(k_stream_collide<D, ST, OCC, TWO, PLAIN>, dim3(grid), dim3(thr), 0, s,
                          (hipEvent_t)cfg.ev0, (hipEvent_t)cfg.ev1, 0u, a);
  else
    k_stream_collide<D, ST, OCC, TWO, PLAIN><<<grid, thr, 0, s>>>(a);
}

template <int D, int ST> static void go_pipe(int grid, const SCArgs &a, const LaunchCfg &cfg, hipStream_t s) {
  if (cfg.ev0)
    hipExtLaunchKernelGGL(k_sc_pipe<D, ST>, dim3(grid), dim3(BN), 0, s, (hipEvent_t)cfg.ev0, (hipEvent_t)cfg.ev1, 0u,
                          a);
  else
    k_sc_pipe<D, ST><<<grid, BN, 0, s>>>(a);
}

int launch_stream_collide(int D, int st, const SCArgs &a, LaunchCfg cfg, void *stream) {
  if (a.n_items <= 0) return 0;
  const int grid = cfg.grid > 0 ? cfg.grid : a.n_items;
  const int thr = cfg.threads > 0 ? cfg.threads : 256;
  hipStream_t s = (hipStream_t)stream;
  if (cfg.pipe == 1) {  // persistent pipelined variant for plain bricks: one node per thread
    ELBM_DISPATCH(D, st, (go_pipe<DD, SS>(grid, a, cfg, s)));
    return ck();
  }
  if (cfg.pipe == 2) {  // plain bricks, one node per thread, at most 128 VGPRs
    ELBM_DISPATCH(D, st, (go_sc<DD, SS, 4, false, true>(grid, BN, a, cfg, s)));
    return ck();
  }
  const bool two = thr == BN / 2;
  if (cfg.occ >= 4 && two)
    ELBM_DISPATCH(D, st, (go_sc<DD, SS, 4, true, false>(grid, thr, a, cfg, s)));
  else if (cfg.occ >= 4)
    ELBM_DISPATCH(D, st, (go_sc<DD, SS, 4, false, false>(grid, thr, a, cfg, s)));
  else if (two)
    ELBM_DISPATCH(D, st, (go_sc<DD, SS, 1, true, false>(grid, thr, a, cfg, s)));
  else
    ELBM_DISPATCH(D, st, (go_sc<DD, SS, 1, false, false>(grid, thr, a, cfg, s)));
  return ck();
}

int launch_gather(int D, int st, const GatherArgs &a, void *stream) {
  if (a.n <= 0) return 0;
  const int grid = (a.n + 255) / 256;
  ELBM_DISPATCH(D, st, (k_gather<DD, SS><<<grid, 256, 0, (hipStream_t)stream>>>(a)));
  return ck();
}

int stage_row_width(int D) { return D == 3 ? stage_width<3>() : stage_width<2>(); }

int couple_lds_stride(int D, int st) {
  const bool dbl = st == ST_F64;
  if (D == 2) return dbl ? lds_stride<2, double>() : lds_stride<2, float>();
  return dbl ? lds_stride<3, double>() : lds_stride<3, float>();
}

// stencil entries of one tile staged in LDS (8 bytes each)
int couple_max_entries() { return 2048; }

int couple_max_rows(int D, int st) {
  const bool dbl = st == ST_F64;
  if (D == 2) return dbl ? couple_rows<2, double>() : couple_rows<2, float>();
  return dbl ? couple_rows<3, double>() : couple_rows<3, float>();
}

int launch_couple(int D, int st, const CoupleArgs &a, void *stream) {
  // one workgroup of two wavefronts per tile (a tile holds one or two brick layers of
  // interface nodes); LDS sized to the largest tile, so several tiles share a CU
  const int ring_blocks = (a.n_ring + COUPLE_THREADS - 1) / COUPLE_THREADS;
  const int grid = a.n_tiles + ring_blocks;
  if (grid <= 0) return 0;
  const int rcap = a.lds_rows > a.lds_items ? a.lds_rows : a.lds_items;
  const size_t lds = (size_t)rcap * couple_lds_stride(D, st) * (st == ST_F64 ? 8 : 4) + (size_t)a.lds_ents * 4;
  ELBM_DISPATCH(D, st, (k_couple<DD, SS><<<grid, COUPLE_THREADS, lds, (hipStream_t)stream>>>(a)));
  return ck();
}

int launch_init(int D, int st, void *pop, const LevelStatic *lev_dev, int level, int nbricks, const int32_t *borg,
                Dims box, const double *rho, const double *u, const double *noise, void *stream) {
  if (nbricks <= 0) return 0;
  ELBM_DISPATCH(D, st,
                (k_init<DD, SS><<<nbricks, BN, 0, (hipStream_t)stream>>>((typename Codec<SS>::S *)pop, lev_dev,
                                                                          level, borg, box, rho, u, noise)));
  return ck();
}

int launch_read(int D, int st, const void *pop, const LevelStatic *lev_dev, int level, int nbricks,
                const int32_t *borg, Dims box, double *rho, double *u, double *gamma, double *f, void *stream) {
  if (nbricks <= 0) return 0;
  ELBM_DISPATCH(D, st,
                (k_read<DD, SS><<<nbricks, BN, 0, (hipStream_t)stream>>>(
                    (const typename Codec<SS>::S *)pop, lev_dev, level, borg, box, rho, u, gamma, f)));
  return ck();
}

int launch_stream_copy(void *dst, const void *src, size_t bytes, int grid, void *stream) {
  const size_t n = bytes / 16;
  if (!n) return 0;
  k_stream_copy<<<grid, 256, 0, (hipStream_t)stream>>>((const float4 *)src, (float4 *)dst, n);
  return ck();
}

int launch_fill_nan(double *p, size_t count, void *stream) {
  if (!count) return 0;
  size_t blocks = (count + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  k_fill_nan<<<(int)blocks, 256, 0, (hipStream_t)stream>>>(p, count);
  return ck();
}

int launch_sample(int D, int st, const void *pop, const LevelStatic *, int, int n, const int32_t *bricks,
                  const int32_t *nodes, double *out, void *stream) {
  if (n <= 0) return 0;
  ELBM_DISPATCH(D, st,
                (k_sample<DD, SS><<<(n + 127) / 128, 128, 0, (hipStream_t)stream>>>(
                    (const typename Codec<SS>::S *)pop, n, bricks, nodes, out)));
  return ck();
}

int launch_reduce(int D, int st, void *const *pops, const LevelStatic *lev_dev, const WorkItem *items, int n_items,
                  double *partials, double *result, void *stream) {
  if (n_items <= 0) return 0;
  ReduceArgs a;
  a.items = items;
  a.n_items = n_items;
  a.lev = lev_dev;
  for (int l = 0; l < MAXL; ++l) a.pop[l] = pops[l];
  a.partials = partials;
  ELBM_DISPATCH(D, st, (k_reduce<DD, SS><<<n_items, BN, 0, (hipStream_t)stream>>>(a)));
  int rc = ck();
  if (rc) return rc;
  k_reduce_final<<<1, 256, 0, (hipStream_t)stream>>>(partials, n_items, result);
  return ck();
}

int launch_force_scatter(int D, float *force, const double *F, int nbricks, const int32_t *borg, Dims box,
                         void *stream) {
  if (nbricks <= 0) return 0;
  if (D == 2) k_force_scatter<2><<<nbricks, BN, 0, (hipStream_t)stream>>>(force, F, borg, box);
  else k_force_scatter<3><<<nbricks, BN, 0, (hipStream_t)stream>>>(force, F, borg, box);
  return ck();
}

int launch_zero(void *p, size_t bytes, void *stream) {
  size_t n = bytes / 4;
  if (!n) return 0;
  size_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  k_zero<<<(int)blocks, 256, 0, (hipStream_t)stream>>>((uint32_t *)p, n);
  return ck();
}

int launch_copy(void *dst, const void *src, size_t bytes, void *stream) {
  return (int)hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, (hipStream_t)stream);
}

}  // namespace elbm
