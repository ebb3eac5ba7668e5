// adjoint.hip -- reverse-mode kernels of the refined KBC coarse step on gfx950.
//
// The paper has no adjoint.  These kernels apply the transpose of the linearisation
// of the discrete coarse step that kernels.hip computes: the collision of Sec. II.A
// (Eq. f_equations, mirror state Eq. f_mirr, stabiliser Eq. gamma_min_approx) with
// the exact-difference forcing of Sec. III.A, the non-equilibrium rescaling
// (Eq. f_neq_rescaling_iso) and four-point reconstruction (Eq. interp) of Sec. III,
// and streaming.  The host runs them tick by tick in reverse order of the
// Sec. III.C schedule on forward states recomputed from checkpoints.  Where
// <dh|dh> = 0 (or the stabiliser is not finite) the forward uses the constant 2,
// which is then not differentiated.  Half-precision storage is differentiated as if
// rounding were the identity.
//
// One tick in reverse:
//   1. collision adjoint over every brick of the arriving levels: lg = (dK/dg)^T lam
//      at stream-collided nodes, 0 elsewhere (plus force-field gradient and the
//      momentum-exchange seed of a drag objective);
//   2. coupling adjoint: reconstructed fine interface nodes write the adjoint of
//      their interpolated (rho~ - 1, u~, n~); coalesced coarse ring nodes add to lg
//      of their fine twin;
//   3. interpolation-point adjoint, one interface pair per launch: the transposed
//      stencil sums the item adjoints, then the reverse of the point's
//      (rho - 1, u, fac (g - f^eq)) adds to lg of the point;
//   4. streaming transpose: lam of the tick's input = lg pulled back along +c_i, plus
//      bounce-back and outflow-copy links.
#include "lbm_device.hpp"

namespace elbm {

// d ln phi(c) / du for the per-axis factor phi(c) = 1 + a(c) of the equilibrium:
// with s = sqrt(1 + 3u^2) = 1 - a(0), sig = s - 1, a(0) = -sig, a(+-1) = 2 sig +- 3u,
// dsig/du = 3u / s.  r[c+1] = 1 / phi(c).
template <typename T> __device__ inline void dlnphi(T u, const T (&a)[3], const T (&r)[3], T (&g)[3]) {
  const T ds = T(3) * u * rcp(T(1) - a[1]);
  g[0] = (T(2) * ds - T(3)) * r[0];
  g[1] = -ds * r[1];
  g[2] = (T(2) * ds + T(3)) * r[2];
}

// Adjoint of q_i(drho, u) = (1 + drho) prod_a phi_a(c_ia) - 1, given t_i = lq_i (1 + q_i):
// ldrho += ir sum t, lu_a += sum_c g_a(c) sum_{i: c_ia = c} t_i.
template <int D, typename T>
__device__ inline void q_adjoint(const T (&t)[nq<D>()], T ir, const T (&g)[3][3], T &ldrho, T (&lu)[3]) {
  T sx[3] = {0, 0, 0}, sy[3] = {0, 0, 0}, sz[3] = {0, 0, 0};
  static_for<0, nq<D>()>([&](auto I) {
    constexpr int i = decltype(I)::value;
    sx[cxo(i) + 1] += t[i];
    sy[cyo(i) + 1] += t[i];
    if (D == 3) sz[czo<D>(i) + 1] += t[i];
  });
  ldrho += ir * ((sx[0] + sx[2]) + sx[1]);
  lu[0] += g[0][0] * sx[0] + g[0][1] * sx[1] + g[0][2] * sx[2];
  lu[1] += g[1][0] * sy[0] + g[1][1] * sy[1] + g[1][2] * sy[2];
  if (D == 3) lu[2] += g[2][0] * sz[0] + g[2][1] * sz[1] + g[2][2] * sz[2];
}

// Adjoint of the shifted equilibrium q(drho, u) alone: adds to ldrho, lu.
template <int D, typename T>
__device__ inline void eq_adjoint(T drho, const T u[3], const T (&lq)[nq<D>()], T &ldrho, T (&lu)[3]) {
  constexpr int Q = nq<D>();
  T a[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  T r[3][3], g[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
  for (int c = 0; c < D; ++c) {
    axis_factors(u[c], a[c]);
#pragma unroll
    for (int k = 0; k < 3; ++k) r[c][k] = rcp(T(1) + a[c][k]);
    dlnphi(u[c], a[c], r[c], g[c]);
  }
  T qxy[9];
  q_table(drho, a, qxy);
  T t[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) t[i] = lq[i] * (T(1) + q_of<D>(qxy, a, i));
  q_adjoint<D, T>(t, rcp(T(1) + drho), g, ldrho, lu);
}

// Reverse of the moments rho - 1 = sum h, u = j / rho: adds (ldrho, lu) into lh.
template <int D, typename T>
__device__ inline void moments_adjoint(T ir, const T u[3], T ldrho, const T (&lu)[3], T (&lh)[nq<D>()]) {
  T lj[3] = {lu[0] * ir, lu[1] * ir, D == 3 ? lu[2] * ir : T(0)};
  ldrho -= ir * (lu[0] * u[0] + lu[1] * u[1] + (D == 3 ? lu[2] * u[2] : T(0)));
  static_for<0, nq<D>()>([&](auto I) {
    constexpr int i = decltype(I)::value;
    T v = ldrho;
    if (cxo(i)) v += T(cxo(i)) * lj[0];
    if (cyo(i)) v += T(cyo(i)) * lj[1];
    if (czo<D>(i)) v += T(czo<D>(i)) * lj[2];
    lh[i] += v;
  });
}

// Reverse of kbc_collide at one node.  h: post-stream shifted populations.  l: on
// entry the adjoint of the post-collision values, on exit the adjoint of h.  lF: the
// adjoint of the force density (level units); the forcing term is always
// differentiated, its derivative wrt F does not vanish at F = 0.
template <int D, typename T>
__device__ inline void kbc_adjoint(const T (&h)[nq<D>()], T (&l)[nq<D>()], T beta, const T F[3], T (&lF)[3]) {
  constexpr int Q = nq<D>();
  T drho, j[3];
  moments<D, T>(h, drho, j);
  const T ir = rcp(T(1) + drho);
  const T u[3] = {j[0] * ir, j[1] * ir, D == 3 ? j[2] * ir : T(0)};
  const T u2[3] = {u[0] + F[0] * ir, u[1] + F[1] * ir, D == 3 ? u[2] + F[2] * ir : T(0)};
  T a[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, a2[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  T r[3][3] = {{1, 1, 1}, {1, 1, 1}, {1, 1, 1}};
#pragma unroll
  for (int c = 0; c < D; ++c) {
    axis_factors(u[c], a[c]);
    axis_factors(u2[c], a2[c]);
#pragma unroll
    for (int k = 0; k < 3; ++k) r[c][k] = rcp(T(1) + a[c][k]);
  }
  // forward recomputation, same arithmetic as kbc_collide
  T q[Q], d[Q];
  {
    T qxy[9];
    q_table(drho, a, qxy);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      q[i] = q_of<D>(qxy, a, i);
      d[i] = h[i] - T(wgt<D>(i)) * q[i];
    }
  }
  auto v = [&](int i) { return d[i]; };
  T N1, N2 = 0, Pxz = 0, Pyz = 0;
  if constexpr (D == 2) {
    N1 = tsum<D, P_XYP, T>(v) - tsum<D, P_XYN, T>(v);
  } else {
    N1 = tsum<D, P_XZP, T>(v) - tsum<D, P_XZN, T>(v);
    N2 = tsum<D, P_YZP, T>(v) - tsum<D, P_YZN, T>(v);
    Pxz = tsum<D, P_MXZP, T>(v) - tsum<D, P_MXZN, T>(v);
    Pyz = tsum<D, P_MYZP, T>(v) - tsum<D, P_MYZN, T>(v);
  }
  const T Pxy = tsum<D, P_MXYP, T>(v) - tsum<D, P_MXYN, T>(v);
  T sX, sY, sZ = 0;
  if (D == 2) {
    sX = T(0.25) * N1;
    sY = -T(0.25) * N1;
  } else {
    const T s6 = T(1.0 / 6.0);
    sX = (T(2) * N1 - N2) * s6;
    sY = (T(2) * N2 - N1) * s6;
    sZ = -(N1 + N2) * s6;
  }
  const T pxy = T(0.25) * Pxy, pxz = T(0.25) * Pxz, pyz = T(0.25) * Pyz;
  auto dsv = [&](int i) -> T {
    const int x = cxo(i), y = cyo(i), z = czo<D>(i);
    const int nz = x * x + y * y + z * z;
    if (nz == 1) return x ? sX : (y ? sY : sZ);
    if (nz == 2) return (z == 0) ? T(x * y) * pxy : ((y == 0) ? T(x * z) * pxz : T(y * z) * pyz);
    return T(0);
  };
  T rxy[9];
#pragma unroll
  for (int cx = 0; cx < 3; ++cx)
#pragma unroll
    for (int cy = 0; cy < 3; ++cy) rxy[cx + 3 * cy] = r[0][cx] * r[1][cy];
  auto ifq = [&](int i) -> T {
    T w = (ir * T(1.0 / wgt<D>(i))) * rxy[(cxo(i) + 1) + 3 * (cyo(i) + 1)];
    if (D == 3) w *= r[2][czo<D>(i) + 1];
    return w;
  };
  const T A = tsum<D, P_SHEAR, T>([&](int i) {
    const T ds = dsv(i);
    return ds * (d[i] - ds) * ifq(i);
  });
  const T B = tsum<D, P_ALL, T>([&](int i) {
    const T dh = d[i] - dsv(i);
    return dh * dh * ifq(i);
  });
  const T ib = rcp(beta);
  T gamma = T(2);
  bool active = false;
  if (B > T(0)) {
    const T g = ib - (T(2) - ib) * (A * rcp(B));
    if (isfinite(g)) {
      gamma = g;
      active = true;
    }
  }
  // ---- reverse
  T g[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, g2[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
  for (int c = 0; c < D; ++c) {
    T r2[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) r2[k] = rcp(T(1) + a2[c][k]);
    dlnphi(u[c], a[c], r[c], g[c]);
    dlnphi(u2[c], a2[c], r2, g2[c]);
  }
  T ldrho = 0, lu[3] = {0, 0, 0}, lu2[3] = {0, 0, 0};
  {  // forcing: out = W q2 + ..., q2 = q(drho, u + F/rho)
    T qxy2[9], t2[Q];
    q_table(drho, a2, qxy2);
#pragma unroll
    for (int i = 0; i < Q; ++i) t2[i] = T(wgt<D>(i)) * l[i] * (T(1) + q_of<D>(qxy2, a2, i));
    q_adjoint<D, T>(t2, ir, g2, ldrho, lu2);
  }
  T lgam = 0;
#pragma unroll
  for (int i = 0; i < Q; ++i) lgam += l[i] * (d[i] - dsv(i));
  lgam *= -beta;
  T lA = 0, lB = 0;
  if (active) {
    const T cc = T(2) - ib, iB = rcp(B);
    lA = -cc * lgam * iB;
    lB = cc * (A * iB) * iB * lgam;
  }
  const T bg = beta * gamma, b2 = T(2) * beta;
  T lds[Q], lq[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const T ds = dsv(i), dh = d[i] - ds, f = ifq(i);
    const T ldh = -bg * l[i] + (lA * ds + T(2) * lB * dh) * f;
    lds[i] = -b2 * l[i] + lA * dh * f - ldh;
    lq[i] = -((lA * ds + lB * dh) * dh) * T(wgt<D>(i)) * f * f;  // d(1/f^eq)/dq = -W / f^eq^2
    l[i] += ldh;                                                  // adjoint of d (direct part)
  }
  // d += S^T lds, S the shear projection d -> ds
  if constexpr (D == 2) {
    T Lx = 0, Ly = 0, Exy = 0;
    static_for<0, Q>([&](auto I) {
      constexpr int i = decltype(I)::value;
      constexpr int x = cxo(i), y = cyo(i);
      if (x * x + y * y == 1) {
        if (x) Lx += lds[i];
        else Ly += lds[i];
      }
      if (x * y) Exy += T(x * y) * lds[i];
    });
    const T n4 = T(0.25) * (Lx - Ly), e4 = T(0.25) * Exy;
    static_for<0, Q>([&](auto I) {
      constexpr int i = decltype(I)::value;
      constexpr int x = cxo(i), y = cyo(i);
      if (x * x - y * y) l[i] += T(x * x - y * y) * n4;
      if (x * y) l[i] += T(x * y) * e4;
    });
  } else {
    T Lx = 0, Ly = 0, Lz = 0, Exy = 0, Exz = 0, Eyz = 0;
    static_for<0, Q>([&](auto I) {
      constexpr int i = decltype(I)::value;
      constexpr int x = cxo(i), y = cyo(i), z = czo<D>(i);
      constexpr int nz = x * x + y * y + z * z;
      if (nz == 1) {
        if (x) Lx += lds[i];
        else if (y) Ly += lds[i];
        else Lz += lds[i];
      }
      if (nz == 2) {
        if (z == 0) Exy += T(x * y) * lds[i];
        else if (y == 0) Exz += T(x * z) * lds[i];
        else Eyz += T(y * z) * lds[i];
      }
    });
    const T s6 = T(1.0 / 6.0);
    const T v1 = (T(2) * Lx - Ly - Lz) * s6, v2 = (T(2) * Ly - Lx - Lz) * s6;
    const T exy = T(0.25) * Exy, exz = T(0.25) * Exz, eyz = T(0.25) * Eyz;
    static_for<0, Q>([&](auto I) {
      constexpr int i = decltype(I)::value;
      constexpr int x = cxo(i), y = cyo(i), z = czo<D>(i);
      if (x * x - z * z) l[i] += T(x * x - z * z) * v1;
      if (y * y - z * z) l[i] += T(y * y - z * z) * v2;
      if (x * y) l[i] += T(x * y) * exy;
      if (x * z) l[i] += T(x * z) * exz;
      if (y * z) l[i] += T(y * z) * eyz;
    });
  }
  // d = h - W q
  {
    T t[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) t[i] = (lq[i] - T(wgt<D>(i)) * l[i]) * (T(1) + q[i]);
    q_adjoint<D, T>(t, ir, g, ldrho, lu);
  }
  // u2 = u + F ir, u = j ir, ir = 1 / (1 + drho)
  T lir = 0;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    lu[c] += lu2[c];
    lF[c] = lu2[c] * ir;
    lir += lu[c] * j[c] + lu2[c] * F[c];
  }
  if (D == 2) lF[2] = T(0);
  ldrho -= ir * ir * lir;
  const T lj[3] = {lu[0] * ir, lu[1] * ir, D == 3 ? lu[2] * ir : T(0)};
  static_for<0, Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    T w = ldrho;
    if (cxo(i)) w += T(cxo(i)) * lj[0];
    if (cyo(i)) w += T(cyo(i)) * lj[1];
    if (czo<D>(i)) w += T(czo<D>(i)) * lj[2];
    l[i] += w;
  });
}

// ---------------------------------------------------------------- 1. collision adjoint
template <int D, int ST> __global__ __launch_bounds__(256) void k_adj_collide(AdjArgs a) {
  using C = Codec<ST>;
  using T = typename C::T;
  constexpr int Q = nq<D>();
  WorkItem w = a.items[blockIdx.x];
  w.brick = __builtin_amdgcn_readfirstlane(w.brick);
  const int wl = __builtin_amdgcn_readfirstlane((int)w.level);
  const int wthr = __builtin_amdgcn_readfirstlane((int)w.thr);
  const LevelStatic &L = a.lev[wl];
  const int32_t *nbp = L.nbr + (size_t)w.brick * 27;
  cptr<int32_t> nbc = cst(L.nbr) + (size_t)w.brick * 27;
  const char *__restrict__ srcb = (const char *)a.src[wl];
  __shared__ uint32_t s_nbo[27];
  if (threadIdx.x < 27) {
    const int nb = nbp[threadIdx.x];
    s_nbo[threadIdx.x] = (uint32_t)(nb < 0 ? 0 : nb) * brick_bytes<D, ST>();
  }
  __syncthreads();
  const T *__restrict__ lam = (const T *)a.lam[wl] + (size_t)w.brick * Q * BN;
  T *__restrict__ lg = (T *)a.lg[wl] + (size_t)w.brick * Q * BN;
  T *__restrict__ lF = a.lF[wl] ? (T *)a.lF[wl] + (size_t)w.brick * D * BN : nullptr;
  const bool seed = wl == a.drag_level;
  for (int n = threadIdx.x; n < BN; n += blockDim.x) {
    const uint8_t cls = L.cls[(size_t)w.brick * BN + n];
    if (!(cls & CLS_FLUID) || (cls & CLS_MODE) < wthr) {
#pragma unroll
      for (int i = 0; i < Q; ++i) lg[i * BN + n] = T(0);
      continue;
    }
    int x, y, z;
    node_xyz<D>(n, x, y, z);
    if (D == 3) z = __builtin_amdgcn_readfirstlane(z);
    T h[Q];
    uint32_t mask = 0;
    {
      uint32_t mid[9], side[9];
      bulk_offsets<D, ST>([&](int q) { return (int)nbc[q]; }, z, mid, side);
      const BulkLane<D> bl(x, y, z);
      const Rsrc rs = buf_rsrc(srcb, (uint32_t)L.nbricks * brick_bytes<D, ST>());
      const bool special = (cls & (CLS_LINKS | CLS_INLET | CLS_OUTFLOW)) != 0;
      if (__builtin_amdgcn_ballot_w64(special) != 0) {
        mask = special ? L.mask[(size_t)w.brick * BN + n] : 0u;
        pull_links<D, ST>(rs, mid, side, bl, [&](int q) { return s_nbo[q]; }, (uint32_t)w.brick * brick_bytes<D, ST>(),
                          x, y, z, n, cls, mask, cst(a.lev) + wl, h);
      } else {
        pull_bulk<D, ST>(rs, mid, side, bl, h);
      }
    }
    T l[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) l[i] = lam[i * BN + n];
    if (seed && (cls & CLS_DRAG)) {  // d/df'_i of the mean momentum exchange 2 c_i f'_i
#pragma unroll
      for (int i = 0; i < Q; ++i)
        if ((mask >> (Q - 1 - i)) & 1u)
          l[i] += T(2.0 * (cxo(i) * a.drag_seed[0] + cyo(i) * a.drag_seed[1] + czo<D>(i) * a.drag_seed[2]));
    }
    T F[3], lFn[3];
    node_force<D, T>(L, w.brick, n, F);
    kbc_adjoint<D, T>(h, l, T(L.beta), F, lFn);
#pragma unroll
    for (int i = 0; i < Q; ++i) lg[i * BN + n] = l[i];
    if (lF)
#pragma unroll
      for (int c = 0; c < D; ++c) lF[c * BN + n] += lFn[c] * T(L.fscale);
  }
}

// ---------------------------------------------------------------- 4. streaming transpose
// Forward: g_i(x) = f'_i(x - c_i), or f'_{Q-1-i}(x) on a bounce-back link, or
// f'_i(x - c_i + o) on an outflow link (o the inward shift), or a constant on an inlet
// link.  For a fluid node y, the node y + c_i never takes population i from y through
// a special link (its source y would be solid or outside the domain), so
//   lam_i(y) = lg_i(y + c_i) + [bounce-back at y] lg_{Q-1-i}(y) + [outflow] lg_i(y + c_i - o).
template <int D, int ST> __global__ __launch_bounds__(256) void k_adj_transpose(AdjArgs a) {
  using C = Codec<ST>;
  using T = typename C::T;
  using Bk = Brick<D>;
  constexpr int Q = nq<D>();
  WorkItem w = a.items[blockIdx.x];
  w.brick = __builtin_amdgcn_readfirstlane(w.brick);
  const int wl = __builtin_amdgcn_readfirstlane((int)w.level);
  const LevelStatic &L = a.lev[wl];
  const AdjLevel &AL = a.alev[wl];
  const int32_t *nbp = L.nbr + (size_t)w.brick * 27;
  const T *__restrict__ lgb = (const T *)a.lg[wl];
  T *__restrict__ out = (T *)a.lam[wl] + (size_t)w.brick * Q * BN;
  auto boff = [&](int code) -> uint32_t {
    const int nb = nbp[code];
    return (uint32_t)(nb < 0 ? AL.zero_brick : nb) * (uint32_t)(Q * BN);
  };
  const uint32_t own = (uint32_t)w.brick * (uint32_t)(Q * BN);
  for (int n = threadIdx.x; n < BN; n += blockDim.x) {
    const uint8_t cls = L.cls[(size_t)w.brick * BN + n];
    if (!(cls & CLS_FLUID)) {
#pragma unroll
      for (int i = 0; i < Q; ++i) out[i * BN + n] = T(0);
      continue;
    }
    int x, y, z;
    node_xyz<D>(n, x, y, z);
    const Lane<D> ln(x, y, z);
    T v[Q];
    static_for<0, Q>([&](auto I) {
      constexpr int i = decltype(I)::value;
      constexpr int o = Q - 1 - i;  // position x + c_i = x - c_o
      v[i] = lgb[boff(ln.code(o)) + (uint32_t)(i * BN + ln.local(o))];
    });
    if (cls & CLS_LINKS) {
      const uint32_t mask = L.mask[(size_t)w.brick * BN + n];
#pragma unroll
      for (int i = 0; i < Q; ++i)
        if ((mask >> (Q - 1 - i)) & 1u) v[i] += lgb[own + (uint32_t)((Q - 1 - i) * BN + n)];
    }
    const uint32_t am = AL.amask ? AL.amask[(size_t)w.brick * BN + n] : 0u;
    if (am) {
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        if (!((am >> i) & 1u)) continue;
        const int sx = x + cxo(i) + L.oshift[0], sy = y + cyo(i) + L.oshift[1],
                  sz = z + czo<D>(i) + L.oshift[2];
        const int code = side<Bk::BX>(sx) + 3 * side<Bk::BY>(sy) + 9 * (D == 3 ? side<Bk::BZ>(sz) : 1);
        const int loc =
            (sx & (Bk::BX - 1)) + Bk::BX * ((sy & (Bk::BY - 1)) + Bk::BY * (D == 3 ? (sz & (Bk::BZ - 1)) : 0));
        v[i] += lgb[boff(code) + (uint32_t)(i * BN + loc)];
      }
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) out[i * BN + n] = v[i];
  }
}

// ---------------------------------------------------------------- 4 + 1 fused
// The streaming transpose of one tick followed, node by node, by the collision adjoint
// of the tick before it (in forward order): the transpose at node y needs only the
// adjoint of the post-stream state at y's neighbours (lg of the later tick, read from
// one buffer), and the collision adjoint at y needs only y's own transposed values, so
// one launch does both and the lam a level collides with need not make a round trip
// through memory before use (it is still stored: the coupling adjoint and the final
// readout read it).  Per level: tpose bit -- the level's lg is transposed into lam;
// coll bit -- the level's collision adjoint runs (on the transposed values when both
// bits are set, else on the stored lam), writing the other lg buffer.
template <int D, int ST> __global__ __launch_bounds__(256) void k_adj_tc(AdjTCArgs a) {
  using C = Codec<ST>;
  using T = typename C::T;
  using Bk = Brick<D>;
  constexpr int Q = nq<D>();
  WorkItem w = a.items[blockIdx.x];
  w.brick = __builtin_amdgcn_readfirstlane(w.brick);
  const int wl = __builtin_amdgcn_readfirstlane((int)w.level);
  const int wthr = __builtin_amdgcn_readfirstlane((int)w.thr);
  const bool tpose = (a.tpose_mask >> wl) & 1u, coll = (a.coll_mask >> wl) & 1u;
  const LevelStatic &L = a.lev[wl];
  const AdjLevel &AL = a.alev[wl];
  const int32_t *nbp = L.nbr + (size_t)w.brick * 27;
  cptr<int32_t> nbc = cst(L.nbr) + (size_t)w.brick * 27;
  // neighbour bricks: byte offsets of the populations (missing -> brick 0, masked by the
  // pull) and element offsets of the adjoint buffer (missing -> the level's zero brick),
  // looked up once per workgroup so that every load of a node's transpose is issued at
  // once rather than after its own index load
  __shared__ uint32_t s_nbo[27], s_nbl[27];
  if (threadIdx.x < 27) {
    const int nb = nbp[threadIdx.x];
    s_nbo[threadIdx.x] = (uint32_t)(nb < 0 ? 0 : nb) * brick_bytes<D, ST>();
    s_nbl[threadIdx.x] = (uint32_t)(nb < 0 ? AL.zero_brick : nb) * (uint32_t)(Q * BN);
  }
  __syncthreads();
  const T *__restrict__ lgb = (const T *)a.lgsrc[wl];
  T *__restrict__ lam = (T *)a.lam[wl] + (size_t)w.brick * Q * BN;
  T *__restrict__ lg = (T *)a.lgdst[wl] + (size_t)w.brick * Q * BN;
  T *__restrict__ lF = a.lF[wl] ? (T *)a.lF[wl] + (size_t)w.brick * D * BN : nullptr;
  const char *__restrict__ srcb = (const char *)a.src[wl];
  auto boff = [&](int code) -> uint32_t { return s_nbl[code]; };
  const uint32_t own = (uint32_t)w.brick * (uint32_t)(Q * BN);
  const bool seed = wl == a.drag_level;
  for (int n = threadIdx.x; n < BN; n += blockDim.x) {
    const uint8_t cls = L.cls[(size_t)w.brick * BN + n];
    const bool fluid = (cls & CLS_FLUID) != 0;
    int x, y, z;
    node_xyz<D>(n, x, y, z);
    T l[Q];
    if (tpose) {
      if (fluid) {
        const Lane<D> ln(x, y, z);
        static_for<0, Q>([&](auto I) {
          constexpr int i = decltype(I)::value;
          constexpr int o = Q - 1 - i;  // position x + c_i = x - c_o
          l[i] = lgb[boff(ln.code(o)) + (uint32_t)(i * BN + ln.local(o))];
        });
        // special links: every load issued (own brick, or a valid neighbour), the
        // terms taken under the link masks
        if (cls & CLS_LINKS) {
          const uint32_t mask = L.mask[(size_t)w.brick * BN + n];
          T v[Q];
#pragma unroll
          for (int i = 0; i < Q; ++i) v[i] = lgb[own + (uint32_t)((Q - 1 - i) * BN + n)];
#pragma unroll
          for (int i = 0; i < Q; ++i)
            if ((mask >> (Q - 1 - i)) & 1u) l[i] += v[i];
        }
        const uint32_t am = AL.amask ? AL.amask[(size_t)w.brick * BN + n] : 0u;
        if (am) {
          T v[Q];
#pragma unroll
          for (int i = 0; i < Q; ++i) {
            const int sx = x + cxo(i) + L.oshift[0], sy = y + cyo(i) + L.oshift[1],
                      sz = z + czo<D>(i) + L.oshift[2];
            const int code = side<Bk::BX>(sx) + 3 * side<Bk::BY>(sy) + 9 * (D == 3 ? side<Bk::BZ>(sz) : 1);
            const int loc =
                (sx & (Bk::BX - 1)) + Bk::BX * ((sy & (Bk::BY - 1)) + Bk::BY * (D == 3 ? (sz & (Bk::BZ - 1)) : 0));
            v[i] = lgb[boff(code) + (uint32_t)(i * BN + loc)];
          }
#pragma unroll
          for (int i = 0; i < Q; ++i)
            if ((am >> i) & 1u) l[i] += v[i];
        }
      } else {
#pragma unroll
        for (int i = 0; i < Q; ++i) l[i] = T(0);
      }
#pragma unroll
      for (int i = 0; i < Q; ++i) lam[i * BN + n] = l[i];
    }
    if (!coll) continue;
    if (!fluid || (cls & CLS_MODE) < wthr) {
#pragma unroll
      for (int i = 0; i < Q; ++i) lg[i * BN + n] = T(0);
      continue;
    }
    if (!tpose) {
#pragma unroll
      for (int i = 0; i < Q; ++i) l[i] = lam[i * BN + n];
    }
    if (D == 3) z = __builtin_amdgcn_readfirstlane(z);
    T h[Q];
    uint32_t mask = 0;
    {
      uint32_t mid[9], side_[9];
      bulk_offsets<D, ST>([&](int q) { return (int)nbc[q]; }, z, mid, side_);
      const BulkLane<D> bl(x, y, z);
      const Rsrc rs = buf_rsrc(srcb, (uint32_t)L.nbricks * brick_bytes<D, ST>());
      const bool special = (cls & (CLS_LINKS | CLS_INLET | CLS_OUTFLOW)) != 0;
      if (__builtin_amdgcn_ballot_w64(special) != 0) {
        mask = special ? L.mask[(size_t)w.brick * BN + n] : 0u;
        pull_links<D, ST>(rs, mid, side_, bl, [&](int q) { return s_nbo[q]; }, (uint32_t)w.brick * brick_bytes<D, ST>(),
                          x, y, z, n, cls, mask, cst(a.lev) + wl, h);
      } else {
        pull_bulk<D, ST>(rs, mid, side_, bl, h);
      }
    }
    if (seed && (cls & CLS_DRAG)) {  // d/df'_i of the mean momentum exchange 2 c_i f'_i
#pragma unroll
      for (int i = 0; i < Q; ++i)
        if ((mask >> (Q - 1 - i)) & 1u)
          l[i] += T(2.0 * (cxo(i) * a.drag_seed[0] + cyo(i) * a.drag_seed[1] + czo<D>(i) * a.drag_seed[2]));
    }
    T F[3], lFn[3];
    node_force<D, T>(L, w.brick, n, F);
    kbc_adjoint<D, T>(h, l, T(L.beta), F, lFn);
#pragma unroll
    for (int i = 0; i < Q; ++i) lg[i * BN + n] = l[i];
    if (lF)
#pragma unroll
      for (int c = 0; c < D; ++c) lF[c * BN + n] += lFn[c] * T(L.fscale);
  }
}

// ---------------------------------------------------------------- 2. coupling adjoint
template <int D, int ST> __global__ __launch_bounds__(64) void k_adj_couple(AdjCoupleArgs A) {
  using C = Codec<ST>;
  using T = typename C::T;
  using V = typename V4<T>::type;
  constexpr int Q = nq<D>();
  constexpr int SW = stage_width<D>();
  const CoupleArgs &a = A.c;
  extern __shared__ __align__(16) unsigned char adj_lds[];
  T *rows = (T *)adj_lds;
  if ((int)blockIdx.x < a.n_tiles) {
    const CTile t = a.tiles[blockIdx.x];
    const V *stage = (const V *)a.stage;
    // entries packed to 4 bytes: tile-local row (16 bits) and the weight in FP16 (the
    // weights are products of -1/16, 9/16 and 1: exact in FP16)
    constexpr int SL = lds_stride<D, T>();
    uint32_t *ents = (uint32_t *)(rows + (size_t)a.lds_rows * SL);
    // rows and entries in rounds of RC per lane, every load of a round issued at once
    // (indices clamped into the tile, which has at least one row and one entry)
    constexpr int NV = SW / 4, RC = 4;
    const int nrow = t.npt * NV;
    for (int k0 = 0; k0 < nrow || k0 < t.ne; k0 += RC * (int)blockDim.x) {
      int ri[RC];
      StencilEntry se[RC];
      V rv[RC];
#pragma unroll
      for (int j = 0; j < RC; ++j) {
        const int k = k0 + j * (int)blockDim.x + (int)threadIdx.x;
        ri[j] = a.tile_rows[t.pt0 + (k < nrow ? k : 0) / NV];
        se[j] = a.sten[t.e0 + (k < t.ne ? k : 0)];
      }
#pragma unroll
      for (int j = 0; j < RC; ++j) {
        const int k = k0 + j * (int)blockDim.x + (int)threadIdx.x;
        rv[j] = stage[(size_t)ri[j] * NV + (k < nrow ? k : 0) % NV];
      }
#pragma unroll
      for (int j = 0; j < RC; ++j) {
        const int k = k0 + j * (int)blockDim.x + (int)threadIdx.x;
        if (k < nrow) ((V *)rows)[(k / NV) * (SL / 4) + k % NV] = rv[j];
        if (k < t.ne) ents[k] = (uint32_t)se[j].slot | ((uint32_t)__half_as_ushort(__float2half_rn(se[j].w)) << 16);
      }
    }
    __syncthreads();
    for (int it = threadIdx.x; it < t.nitem; it += blockDim.x) {
      const CItem c = a.items[t.item0 + it];
      T acc[SW];
#pragma unroll
      for (int v = 0; v < SW; ++v) acc[v] = 0;
      for (int e = c.a - t.e0; e < c.a - t.e0 + c.b; ++e) {
        const uint32_t s = ents[e];
        const T w = T(__half2float(__ushort_as_half((uint16_t)(s >> 16))));
        const V *row = (const V *)(rows + (s & 0xffffu) * SL);
#pragma unroll
        for (int v = 0; v < SW / 4; ++v) {
          const V r = row[v];
          acc[4 * v + 0] = fma(w, r.x, acc[4 * v + 0]);
          acc[4 * v + 1] = fma(w, r.y, acc[4 * v + 1]);
          acc[4 * v + 2] = fma(w, r.z, acc[4 * v + 2]);
          acc[4 * v + 3] = fma(w, r.w, acc[4 * v + 3]);
        }
      }
      const T u[3] = {acc[1], acc[2], D == 3 ? acc[3] : T(0)};
      T q[Q], h[Q];
      eq_dev<D, T>(acc[0], u, q);
#pragma unroll
      for (int i = 0; i < Q; ++i) h[i] = acc[1 + D + i] + T(wgt<D>(i)) * q[i];
      const LevelStatic &L = a.lev[c.level];
      const size_t base = (size_t)c.brick * Q * BN + c.node;
      const T *lam = (const T *)A.lam[c.level] + base;
      T l[Q];
#pragma unroll
      for (int i = 0; i < Q; ++i) l[i] = lam[i * BN];
      T F[3], lFn[3];
      node_force<D, T>(L, c.brick, c.node, F);
      kbc_adjoint<D, T>(h, l, T(L.beta), F, lFn);
      if (A.lF[c.level]) {
        T *lF = (T *)A.lF[c.level] + (size_t)c.brick * D * BN + c.node;
#pragma unroll
        for (int k = 0; k < D; ++k) lF[k * BN] += lFn[k] * T(L.fscale);
      }
      // h = n~ + W q(rho~ - 1, u~)
      T lq[Q], lr = 0, lu[3] = {0, 0, 0};
#pragma unroll
      for (int i = 0; i < Q; ++i) lq[i] = T(wgt<D>(i)) * l[i];
      eq_adjoint<D, T>(acc[0], u, lq, lr, lu);
      T *o = (T *)A.astage + (size_t)(t.item0 + it) * SW;
      o[0] = lr;
#pragma unroll
      for (int k = 0; k < D; ++k) o[1 + k] = lu[k];
#pragma unroll
      for (int i = 0; i < Q; ++i) o[1 + D + i] = l[i];
      if (D == 3) o[31] = T(0);
    }
    return;
  }
  // coarse ring node: g = f^eq + fac (g_twin - f^eq), f^eq at the twin's moments
  const int t = ((int)blockIdx.x - a.n_tiles) * blockDim.x + threadIdx.x;
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
  const T u[3] = {j[0] * ir, j[1] * ir, j[2] * ir};
  T q[Q], hr[Q];
  eq_dev<D, T>(drho, u, q);
  const T fac = T(a.pairs[c.level].fac_cp);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const T heq = T(wgt<D>(i)) * q[i];
    hr[i] = heq + fac * (h[i] - heq);
  }
  const LevelStatic &L = a.lev[c.level];
  const T *lam = (const T *)A.lam[c.level] + (size_t)c.brick * Q * BN + c.node;
  T l[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) l[i] = lam[i * BN];
  T F[3], lFn[3];
  node_force<D, T>(L, c.brick, c.node, F);
  kbc_adjoint<D, T>(hr, l, T(L.beta), F, lFn);
  if (A.lF[c.level]) {
    T *lF = (T *)A.lF[c.level] + (size_t)c.brick * D * BN + c.node;
#pragma unroll
    for (int k = 0; k < D; ++k) lF[k * BN] += lFn[k] * T(L.fscale);
  }
  T lh[Q], lq[Q], lr = 0, lu[3] = {0, 0, 0};
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    lh[i] = fac * l[i];
    lq[i] = (T(1) - fac) * T(wgt<D>(i)) * l[i];
  }
  eq_adjoint<D, T>(drho, u, lq, lr, lu);
  moments_adjoint<D, T>(ir, u, lr, lu, lh);
  T *lg = (T *)A.lg[fl] + (size_t)c.a * Q * BN + c.b;
#pragma unroll
  for (int i = 0; i < Q; ++i) lg[i * BN] += lh[i];
}

// ---------------------------------------------------------------- 3. point adjoint
template <int D, int ST> __global__ __launch_bounds__(128) void k_adj_points(AdjPointArgs a) {
  using C = Codec<ST>;
  using T = typename C::T;
  constexpr int Q = nq<D>();
  constexpr int SW = stage_width<D>();
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.n) return;
  const GPoint g = a.pts[p];
  T lrow[SW];
#pragma unroll
  for (int v = 0; v < SW; ++v) lrow[v] = 0;
  // the transposed stencil in rounds of four entries, their loads issued together (the
  // index clamped to the last entry; an entry past the end adds with weight zero)
  const int e0 = a.tofs[g.slot], e1 = a.tofs[g.slot + 1];
  for (int e = e0; e < e1; e += 4) {
    StencilEntry s[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) s[k] = a.tsten[e + k < e1 ? e + k : e1 - 1];
    T r[4][SW];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int v = 0; v < SW; ++v) r[k][v] = ((const T *)a.astage)[(size_t)s[k].slot * SW + v];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const T w = e + k < e1 ? T(s[k].w) : T(0);
#pragma unroll
      for (int v = 0; v < SW; ++v) lrow[v] = fma(w, r[k][v], lrow[v]);
    }
  }
  const LevelStatic &L = a.lev[g.level];
  const char *srcb = (const char *)a.src[g.level];
  const int32_t *nb = L.nbr + (size_t)g.brick * 27;
  auto boff = [&](int code) { return (uint32_t)nb[code] * brick_bytes<D, ST>(); };
  int x, y, z;
  node_xyz<D>(g.node, x, y, z);
  const Lane<D> ln(x, y, z);
  T h[Q];
  pull_plain<D, ST>(srcb, boff, ln, h);
  T drho, j[3];
  moments<D, T>(h, drho, j);
  const T ir = rcp(T(1) + drho);
  const T u[3] = {j[0] * ir, j[1] * ir, j[2] * ir};
  const PairStatic &P = a.pairs[g.pair];
  const T fac = (g.level == P.parent) ? T(P.fac_pc) : T(1);
  // row = (drho, u, fac (h - W q(drho, u)))
  T lh[Q], lq[Q], lr = lrow[0], lu[3] = {lrow[1], lrow[2], D == 3 ? lrow[3] : T(0)};
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    lh[i] = fac * lrow[1 + D + i];
    lq[i] = -T(wgt<D>(i)) * lh[i];
  }
  eq_adjoint<D, T>(drho, u, lq, lr, lu);
  moments_adjoint<D, T>(ir, u, lr, lu, lh);
  T *lg = (T *)a.lg[g.level] + (size_t)g.brick * Q * BN + g.node;
#pragma unroll
  for (int i = 0; i < Q; ++i) lg[i * BN] += lh[i];
}

// ---------------------------------------------------------------- objective: kinetic energy
// J = 1/2 sum_l sum_x w |j - F/2|^2 / rho at the final state (owned-volume weights w);
// seeds lam = dJ/df and the force-field gradient with dJ/dF.
template <int D, int ST> __global__ __launch_bounds__(256) void k_adj_ke(AdjKEArgs a) {
  using C = Codec<ST>;
  using T = typename C::T;
  constexpr int Q = nq<D>();
  __shared__ double s[4];
  const WorkItem w = a.items[blockIdx.x];
  const LevelStatic &L = a.lev[w.level];
  const int n = threadIdx.x;
  const uint8_t cls = L.cls[(size_t)w.brick * BN + n];
  const typename C::S *p = (const typename C::S *)a.pop[w.level] + (size_t)w.brick * Q * BN + n;
  T *lam = (T *)a.lam[w.level] + (size_t)w.brick * Q * BN + n;
  double J = 0;
  if (cls & CLS_FLUID) {
    double drho = 0, j[3] = {0, 0, 0};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const double hi = (double)C::ld(p + i * BN, T(wgt<D>(i)));
      drho += hi;
      j[0] += cxo(i) * hi;
      j[1] += cyo(i) * hi;
      j[2] += czo<D>(i) * hi;
    }
    double F[3];
    node_force<D, double>(L, w.brick, n, F);
    const double rho = 1.0 + drho, wt = (double)L.weight[(size_t)w.brick * BN + n];
    const double pm[3] = {j[0] - 0.5 * F[0], j[1] - 0.5 * F[1], j[2] - 0.5 * F[2]};
    const double p2 = pm[0] * pm[0] + pm[1] * pm[1] + pm[2] * pm[2];
    J = 0.5 * wt * p2 / rho;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const double pc = pm[0] * cxo(i) + pm[1] * cyo(i) + pm[2] * czo<D>(i);
      lam[i * BN] = T(wt * (pc / rho - 0.5 * p2 / (rho * rho)));
    }
    if (a.lF[w.level]) {
      T *lF = (T *)a.lF[w.level] + (size_t)w.brick * D * BN + n;
      for (int c = 0; c < D; ++c) lF[c * BN] += T(-0.5 * wt * pm[c] / rho * L.fscale);
    }
  } else {
#pragma unroll
    for (int i = 0; i < Q; ++i) lam[i * BN] = T(0);
  }
  for (int off = 32; off > 0; off >>= 1) J += __shfl_down(J, off, 64);
  if ((n & 63) == 0) s[n >> 6] = J;
  __syncthreads();
  if (n < 5) a.partials[(size_t)blockIdx.x * 5 + n] = n == 0 ? ((s[0] + s[1]) + (s[2] + s[3])) : 0.0;
}

// ---------------------------------------------------------------- readout of adjoint fields
template <int D, int ST>
__global__ __launch_bounds__(256) void k_adj_read(const void *lamv, const void *lFv, const LevelStatic *lev,
                                                  int level, const int32_t *borg, Dims box, double *lam_out,
                                                  double *lF_out) {
  using T = typename Codec<ST>::T;
  constexpr int Q = nq<D>();
  const int b = blockIdx.x, n = threadIdx.x;
  const LevelStatic &L = lev[level];
  if (!(L.cls[(size_t)b * BN + n] & CLS_FLUID)) return;
  int x, y, z;
  node_xyz<D>(n, x, y, z);
  const int64_t X = borg[3 * b] + x, Y = borg[3 * b + 1] + y, Z = borg[3 * b + 2] + z;
  if (X >= box.n[0] || Y >= box.n[1] || Z >= box.n[2]) return;
  const int64_t tot = box.n[0] * box.n[1] * box.n[2];
  const int64_t k = X + box.n[0] * (Y + box.n[1] * Z);
  if (lam_out && lamv) {
    const T *l = (const T *)lamv + (size_t)b * Q * BN + n;
    for (int i = 0; i < Q; ++i) lam_out[(int64_t)i * tot + k] = (double)l[i * BN];
  }
  if (lF_out && lFv) {
    const T *l = (const T *)lFv + (size_t)b * D * BN + n;
    for (int c = 0; c < D; ++c) lF_out[(int64_t)c * tot + k] = (double)l[c * BN];
  }
}

// gradient wrt the initial velocity through f = f^eq(rho0, u0) (1 + noise) (the
// initialisation of k_init), from the adjoint of the initial state
template <int D, int ST>
__global__ __launch_bounds__(256) void k_adj_velocity(const void *lamv, const LevelStatic *lev, int level,
                                                      const int32_t *borg, Dims box, const double *rho,
                                                      const double *u, const double *noise, double *out) {
  using T = typename Codec<ST>::T;
  constexpr int Q = nq<D>();
  const int b = blockIdx.x, n = threadIdx.x;
  const LevelStatic &L = lev[level];
  if (!(L.cls[(size_t)b * BN + n] & CLS_FLUID)) return;
  int x, y, z;
  node_xyz<D>(n, x, y, z);
  const int64_t X = borg[3 * b] + x, Y = borg[3 * b + 1] + y, Z = borg[3 * b + 2] + z;
  if (X >= box.n[0] || Y >= box.n[1] || Z >= box.n[2]) return;
  const int64_t tot = box.n[0] * box.n[1] * box.n[2];
  const int64_t k = X + box.n[0] * (Y + box.n[1] * Z);
  const T *l = (const T *)lamv + (size_t)b * Q * BN + n;
  const double uu[3] = {u[k], u[tot + k], D == 3 ? u[2 * tot + k] : 0.0};
  double lq[Q], lr = 0, lu[3] = {0, 0, 0};
  for (int i = 0; i < Q; ++i) lq[i] = (double)l[i * BN] * wgt<D>(i) * (noise ? 1.0 + noise[(int64_t)i * tot + k] : 1.0);
  eq_adjoint<D, double>(rho[k] - 1.0, uu, lq, lr, lu);
  for (int c = 0; c < D; ++c) out[(int64_t)c * tot + k] = lu[c];
}

__global__ void k_reduce_final5(const double *partials, int n, double *out) {
  __shared__ double s[256];
  double v = 0;
  for (int i = threadIdx.x; i < n; i += 256) v += partials[(size_t)i * 5];
  s[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = s[0];
}

// ---------------------------------------------------------------- launchers
static int ack() { return (int)hipGetLastError(); }

#define ELBM_ADJ_DISPATCH(D, st, CALL)                             \
  do {                                                             \
    if (D == 2) {                                                  \
      constexpr int DD = 2;                                        \
      switch (st) {                                                \
        case ST_F64: { constexpr int SS = ST_F64; CALL; } break;   \
        case ST_F32: { constexpr int SS = ST_F32; CALL; } break;   \
        case ST_F16S: { constexpr int SS = ST_F16S; CALL; } break; \
        default: { constexpr int SS = ST_BF16S; CALL; } break;     \
      }                                                            \
    } else {                                                       \
      constexpr int DD = 3;                                        \
      switch (st) {                                                \
        case ST_F64: { constexpr int SS = ST_F64; CALL; } break;   \
        case ST_F32: { constexpr int SS = ST_F32; CALL; } break;   \
        case ST_F16S: { constexpr int SS = ST_F16S; CALL; } break; \
        default: { constexpr int SS = ST_BF16S; CALL; } break;     \
      }                                                            \
    }                                                              \
  } while (0)

int launch_adj_collide(int D, int st, const AdjArgs &a, void *stream) {
  if (a.n_items <= 0) return 0;
  ELBM_ADJ_DISPATCH(D, st, (k_adj_collide<DD, SS><<<a.n_items, 256, 0, (hipStream_t)stream>>>(a)));
  return ack();
}

int launch_adj_transpose(int D, int st, const AdjArgs &a, void *stream) {
  if (a.n_items <= 0) return 0;
  ELBM_ADJ_DISPATCH(D, st, (k_adj_transpose<DD, SS><<<a.n_items, 256, 0, (hipStream_t)stream>>>(a)));
  return ack();
}

int launch_adj_tc(int D, int st, const AdjTCArgs &a, void *stream) {
  if (a.n_items <= 0) return 0;
  ELBM_ADJ_DISPATCH(D, st, (k_adj_tc<DD, SS><<<a.n_items, 256, 0, (hipStream_t)stream>>>(a)));
  return ack();
}

int launch_adj_couple(int D, int st, const AdjCoupleArgs &a, void *stream) {
  const int grid = a.c.n_tiles + (a.c.n_ring + 63) / 64;
  if (grid <= 0) return 0;
  const size_t lds = (size_t)a.c.lds_rows * couple_lds_stride(D, st) * (st == ST_F64 ? 8 : 4) + (size_t)a.c.lds_ents * 4;
  ELBM_ADJ_DISPATCH(D, st, (k_adj_couple<DD, SS><<<grid, 64, lds, (hipStream_t)stream>>>(a)));
  return ack();
}

int launch_adj_points(int D, int st, const AdjPointArgs &a, void *stream) {
  if (a.n <= 0) return 0;
  ELBM_ADJ_DISPATCH(D, st, (k_adj_points<DD, SS><<<(a.n + 127) / 128, 128, 0, (hipStream_t)stream>>>(a)));
  return ack();
}

int launch_adj_ke(int D, int st, const AdjKEArgs &a, double *result, void *stream) {
  if (a.n_items <= 0) return 0;
  ELBM_ADJ_DISPATCH(D, st, (k_adj_ke<DD, SS><<<a.n_items, 256, 0, (hipStream_t)stream>>>(a)));
  k_reduce_final5<<<1, 256, 0, (hipStream_t)stream>>>(a.partials, a.n_items, result);
  return ack();
}

int launch_adj_read(int D, int st, const void *lam, const void *lF, const LevelStatic *lev_dev, int level,
                    int nbricks, const int32_t *borg, Dims box, double *lam_out, double *lF_out, void *stream) {
  if (nbricks <= 0) return 0;
  ELBM_ADJ_DISPATCH(D, st,
                    (k_adj_read<DD, SS><<<nbricks, BN, 0, (hipStream_t)stream>>>(lam, lF, lev_dev, level, borg, box,
                                                                              lam_out, lF_out)));
  return ack();
}

int launch_adj_velocity(int D, int st, const void *lam, const LevelStatic *lev_dev, int level, int nbricks,
                        const int32_t *borg, Dims box, const double *rho, const double *u, const double *noise,
                        double *out, void *stream) {
  if (nbricks <= 0) return 0;
  ELBM_ADJ_DISPATCH(D, st,
                    (k_adj_velocity<DD, SS><<<nbricks, BN, 0, (hipStream_t)stream>>>(lam, lev_dev, level, borg, box,
                                                                                  rho, u, noise, out)));
  return ack();
}

}  // namespace elbm
