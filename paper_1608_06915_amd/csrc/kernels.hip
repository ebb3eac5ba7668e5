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
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "elbm_dev.hpp"

namespace elbm {

// ---------------------------------------------------------------- lattice constants
__host__ __device__ constexpr int cxo(int i) { return i % 3 - 1; }
__host__ __device__ constexpr int cyo(int i) { return (i / 3) % 3 - 1; }
template <int D> __host__ __device__ constexpr int czo(int i) { return D == 3 ? i / 9 - 1 : 0; }
template <int D> __host__ __device__ constexpr int nq() { return D == 2 ? 9 : 27; }
__host__ __device__ constexpr double w1(int c) { return c == 0 ? 2.0 / 3.0 : 1.0 / 6.0; }
template <int D> __host__ __device__ constexpr double wgt(int i) {
  return w1(cxo(i)) * w1(cyo(i)) * (D == 3 ? w1(czo<D>(i)) : 1.0);
}

// ---------------------------------------------------------------- storage codecs
template <int ST> struct Codec;
template <> struct Codec<ST_F64> {
  typedef double S;
  typedef double T;
  __device__ static inline T ld(const S *p, T w) { return *p - w; }
  __device__ static inline void st(S *p, T h, T w) { *p = w + h; }
};
template <> struct Codec<ST_F32> {
  typedef float S;
  typedef float T;
  __device__ static inline T ld(const S *p, T w) { return *p - w; }
  __device__ static inline void st(S *p, T h, T w) { *p = w + h; }
};
template <> struct Codec<ST_F16S> {
  typedef uint16_t S;
  typedef float T;
  __device__ static inline T ld(const S *p, T) { return __half2float(__ushort_as_half(*p)); }
  __device__ static inline void st(S *p, T h, T) { *p = __half_as_ushort(__float2half_rn(h)); }
};
template <> struct Codec<ST_BF16S> {
  typedef uint16_t S;
  typedef float T;
  __device__ static inline T ld(const S *p, T) { return __uint_as_float(((uint32_t)*p) << 16); }
  __device__ static inline void st(S *p, T h, T) {
    uint32_t b = __float_as_uint(h);
    if ((b & 0x7fffffffu) > 0x7f800000u) {
      *p = (uint16_t)0x7fc0u;
    } else {
      b += 0x7fffu + ((b >> 16) & 1u);  // round to nearest, ties to even
      *p = (uint16_t)(b >> 16);
    }
  }
};

// FP32 uses the hardware reciprocal and square root (about 1 ulp); FP64 keeps IEEE
// division and square root.
__device__ inline float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double rcp(double x) { return 1.0 / x; }
__device__ inline float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ inline double sqrt_(double x) { return sqrt(x); }

// ---------------------------------------------------------------- equilibrium
// per-axis a(c) = phi(c) - 1 for c = -1, 0, +1 (index c+1)
template <typename T> __device__ inline void axis_factors(T u, T a[3]) {
  T t = T(3) * u * u;
  T sig = t * rcp(T(1) + sqrt_(T(1) + t));
  a[0] = T(2) * sig - T(3) * u;
  a[1] = -sig;
  a[2] = T(2) * sig + T(3) * u;
}

// partial products over x and y: qxy[cx+1 + 3(cy+1)] = (1+drho)(1+ax)(1+ay) - 1
template <typename T> __device__ inline void q_table(T drho, const T (&a)[3][3], T (&qxy)[9]) {
#pragma unroll
  for (int cx = 0; cx < 3; ++cx) {
    const T qx = fma(drho, a[0][cx], drho + a[0][cx]);
#pragma unroll
    for (int cy = 0; cy < 3; ++cy) qxy[cx + 3 * cy] = fma(qx, a[1][cy], qx + a[1][cy]);
  }
}
// q_i = (1 + drho) prod_a phi_a(c_ia) - 1, so that f_i^eq - W_i = W_i q_i
template <int D, typename T> __device__ inline T q_of(const T (&qxy)[9], const T (&a)[3][3], int i) {
  T v = qxy[(cxo(i) + 1) + 3 * (cyo(i) + 1)];
  if (D == 3) {
    const T b = a[2][czo<D>(i) + 1];
    v = fma(v, b, v + b);
  }
  return v;
}

template <int D, typename T> __device__ inline void eq_dev(T drho, const T u[3], T (&q)[nq<D>()]) {
  T a[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  axis_factors(u[0], a[0]);
  axis_factors(u[1], a[1]);
  if (D == 3) axis_factors(u[2], a[2]);
  T qxy[9];
  q_table(drho, a, qxy);
#pragma unroll
  for (int i = 0; i < nq<D>(); ++i) q[i] = q_of<D>(qxy, a, i);
}

template <int D, typename T> __device__ inline void moments(const T (&h)[nq<D>()], T &drho, T (&j)[3]) {
  drho = 0;
  j[0] = j[1] = j[2] = 0;
#pragma unroll
  for (int i = 0; i < nq<D>(); ++i) {
    drho += h[i];
    if (cxo(i) == 1) j[0] += h[i];
    if (cxo(i) == -1) j[0] -= h[i];
    if (cyo(i) == 1) j[1] += h[i];
    if (cyo(i) == -1) j[1] -= h[i];
    if (D == 3 && czo<D>(i) == 1) j[2] += h[i];
    if (D == 3 && czo<D>(i) == -1) j[2] -= h[i];
  }
}

// ---------------------------------------------------------------- KBC collision
// Post-collision h' = h - beta (2 ds + gamma dh) (Eq. f_equations with Eq. f_mirr),
// gamma from Eq. gamma_min_approx, plus the exact-difference forcing of Sec. III.A.
// h is overwritten by the deviation d = h - (f^eq - W); the post-collision value of
// population i is handed to st(i, h'_i).  F: force density in level units.
template <int D, typename T, typename Store>
__device__ inline T kbc_collide(T (&h)[nq<D>()], T beta, const T F[3], bool has_force, Store st) {
  constexpr int Q = nq<D>();
  T drho, j[3];
  moments<D, T>(h, drho, j);
  const T ir = rcp(T(1) + drho);
  const T u[3] = {j[0] * ir, j[1] * ir, D == 3 ? j[2] * ir : T(0)};
  T a[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  axis_factors(u[0], a[0]);
  axis_factors(u[1], a[1]);
  if (D == 3) axis_factors(u[2], a[2]);
  {
    T qxy[9];
    q_table(drho, a, qxy);
#pragma unroll
    for (int i = 0; i < Q; ++i) h[i] -= T(wgt<D>(i)) * q_of<D>(qxy, a, i);
  }
  // deviatoric second moments of d
  T N1 = 0, N2 = 0, Pxy = 0, Pxz = 0, Pyz = 0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int x = cxo(i), y = cyo(i), z = czo<D>(i);
    const T d = h[i];
    if (D == 2) {
      const int nn = x * x - y * y;
      if (nn == 1) N1 += d;
      if (nn == -1) N1 -= d;
    } else {
      const int a1 = x * x - z * z, a2 = y * y - z * z;
      if (a1 == 1) N1 += d;
      if (a1 == -1) N1 -= d;
      if (a2 == 1) N2 += d;
      if (a2 == -1) N2 -= d;
      if (x * z == 1) Pxz += d;
      if (x * z == -1) Pxz -= d;
      if (y * z == 1) Pyz += d;
      if (y * z == -1) Pyz -= d;
    }
    if (x * y == 1) Pxy += d;
    if (x * y == -1) Pxy -= d;
  }
  // shear-part values (natural-moment basis, trace in h)
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
  // entropic scalar products <ds|dh>, <dh|dh> with weight 1/f^eq = (1/(rho W)) prod 1/phi
  T A = 0, B = 0;
  {
    T rxy[9], rz[3] = {1, 1, 1};
#pragma unroll
    for (int cx = 0; cx < 3; ++cx) {
      const T rx = rcp(T(1) + a[0][cx]);
#pragma unroll
      for (int cy = 0; cy < 3; ++cy) rxy[cx + 3 * cy] = rx * rcp(T(1) + a[1][cy]);
    }
    if (D == 3)
#pragma unroll
      for (int c = 0; c < 3; ++c) rz[c] = rcp(T(1) + a[2][c]);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const T ds = dsv(i);
      const T dh = h[i] - ds;
      T ifq = (ir * T(1.0 / wgt<D>(i))) * rxy[(cxo(i) + 1) + 3 * (cyo(i) + 1)];
      if (D == 3) ifq *= rz[czo<D>(i) + 1];
      const T dhw = dh * ifq;
      A = fma(ds, dhw, A);
      B = fma(dh, dhw, B);
    }
  }
  const T ib = rcp(beta);
  T gamma = T(2);
  if (B > T(0)) {
    const T g = ib - (T(2) - ib) * (A * rcp(B));
    if (isfinite(g)) gamma = g;
  }
  const T b2 = T(2) * beta, bg = beta * gamma;
  T qxy[9];
  q_table(drho, a, qxy);
  if (has_force) {
    const T u2[3] = {u[0] + F[0] * ir, u[1] + F[1] * ir, D == 3 ? u[2] + F[2] * ir : T(0)};
    T a2[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    axis_factors(u2[0], a2[0]);
    axis_factors(u2[1], a2[1]);
    if (D == 3) axis_factors(u2[2], a2[2]);
    T qxy2[9];
    q_table(drho, a2, qxy2);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const T ds = dsv(i), d = h[i];
      const T q = q_of<D>(qxy, a, i);
      const T q2 = q_of<D>(qxy2, a2, i);
      st(i, T(wgt<D>(i)) * q2 + (d - b2 * ds - bg * (d - ds)));
    }
  } else {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const T ds = dsv(i), d = h[i];
      st(i, T(wgt<D>(i)) * q_of<D>(qxy, a, i) + (d - b2 * ds - bg * (d - ds)));
    }
  }
  return gamma;
}

template <int D, typename T> __device__ inline void node_force(const LevelStatic &L, int brick, int n, T F[3]) {
  F[0] = T(L.F[0]);
  F[1] = T(L.F[1]);
  F[2] = T(L.F[2]);
  if (L.force) {
    const float *fp = L.force + (size_t)brick * D * BN + n;
#pragma unroll
    for (int a = 0; a < D; ++a) F[a] += T(fp[a * BN]) * T(L.fscale);
  }
}

// ---------------------------------------------------------------- pull streaming
// Sources are addressed as 32-bit byte offsets from the level's population buffer
// (an SGPR base): offset = brick_offset[neighbour code] + (i*BN + local node)*size.
template <int B> __device__ inline int side(int s) { return s < 0 ? 0 : (s >= B ? 2 : 1); }

template <int D> struct Lane {
  // per source displacement k = c+1 along each axis: neighbour code part, local index part
  int xb[3], xl[3], yzb[9], yzl[9];
  __device__ inline Lane(int x, int y, int z) {
    using Bk = Brick<D>;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int sx = x + 1 - k;
      xb[k] = side<Bk::BX>(sx);
      xl[k] = sx & (Bk::BX - 1);
    }
#pragma unroll
    for (int ky = 0; ky < 3; ++ky)
#pragma unroll
      for (int kz = 0; kz < 3; ++kz) {
        const int sy = y + 1 - ky;
        const int sz = D == 3 ? z + 1 - kz : 0;
        yzb[ky + 3 * kz] = 3 * side<Bk::BY>(sy) + 9 * (D == 3 ? side<Bk::BZ>(sz) : 1);
        yzl[ky + 3 * kz] = Bk::BX * ((sy & (Bk::BY - 1)) + Bk::BY * (D == 3 ? (sz & (Bk::BZ - 1)) : 0));
      }
  }
  __device__ inline int code(int i) const {
    return xb[cxo(i) + 1] + yzb[(cyo(i) + 1) + 3 * (czo<D>(i) + 1)];
  }
  __device__ inline int local(int i) const {
    return xl[cxo(i) + 1] + yzl[(cyo(i) + 1) + 3 * (czo<D>(i) + 1)];
  }
};

template <int D, int ST, typename OFF>
__device__ inline void pull_plain(const char *__restrict__ srcb, OFF boff, const Lane<D> &ln,
                                  typename Codec<ST>::T (&h)[nq<D>()]) {
  using C = Codec<ST>;
  using S = typename C::S;
  using T = typename C::T;
#pragma unroll
  for (int i = 0; i < nq<D>(); ++i) {
    const uint32_t off = boff(ln.code(i)) + (uint32_t)((i * BN + ln.local(i)) * (int)sizeof(S));
    h[i] = C::ld((const S *)(srcb + off), T(wgt<D>(i)));
  }
}

template <int D, int ST, typename OFF>
__device__ inline void pull_special(const char *__restrict__ srcb, OFF boff, const Lane<D> &ln, int n,
                                    uint8_t cls, uint32_t mask, const LevelStatic &L,
                                    typename Codec<ST>::T (&h)[nq<D>()]) {
  using C = Codec<ST>;
  using S = typename C::S;
  using T = typename C::T;
  using Bk = Brick<D>;
  constexpr int Q = nq<D>();
  const uint32_t own = boff(13);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const bool hit = (mask >> i) & 1u;
    if (hit && (cls & CLS_LINKS)) {  // halfway bounce-back: own node, opposite velocity
      h[i] = C::ld((const S *)(srcb + own + (uint32_t)(((Q - 1 - i) * BN + n) * (int)sizeof(S))),
                   T(wgt<D>(Q - 1 - i)));
      continue;
    }
    if (hit && (cls & CLS_INLET)) {
      h[i] = T(L.hin[i]);
      continue;
    }
    if (hit && (cls & CLS_OUTFLOW)) {  // zero gradient: value one node upstream
      int x = n & (Bk::BX - 1), y = (n >> Bk::LX) & (Bk::BY - 1), z = D == 3 ? n >> (Bk::LX + Bk::LY) : 0;
      const int sx = x - cxo(i) - L.oshift[0], sy = y - cyo(i) - L.oshift[1], sz = z - czo<D>(i) - L.oshift[2];
      const int code = side<Bk::BX>(sx) + 3 * side<Bk::BY>(sy) + 9 * (D == 3 ? side<Bk::BZ>(sz) : 1);
      const int loc =
          (sx & (Bk::BX - 1)) + Bk::BX * ((sy & (Bk::BY - 1)) + Bk::BY * (D == 3 ? (sz & (Bk::BZ - 1)) : 0));
      h[i] = C::ld((const S *)(srcb + boff(code) + (uint32_t)((i * BN + loc) * (int)sizeof(S))), T(wgt<D>(i)));
      continue;
    }
    const uint32_t off = boff(ln.code(i)) + (uint32_t)((i * BN + ln.local(i)) * (int)sizeof(S));
    h[i] = C::ld((const S *)(srcb + off), T(wgt<D>(i)));
  }
}

template <int D> __device__ inline void node_xyz(int n, int &x, int &y, int &z) {
  using Bk = Brick<D>;
  x = n & (Bk::BX - 1);
  y = (n >> Bk::LX) & (Bk::BY - 1);
  z = D == 3 ? (n >> (Bk::LX + Bk::LY)) : 0;
}

__device__ inline int xcd_perm(int b, int G) {
  // workgroups are dealt round-robin to the 8 XCDs; give each XCD a contiguous range
  return (b & 7) * (G >> 3) + (b >> 3);
}

template <int D, int ST> __device__ constexpr uint32_t brick_bytes() {
  return (uint32_t)(nq<D>() * BN * sizeof(typename Codec<ST>::S));
}

// ---------------------------------------------------------------- stream-collide
// OCC: minimum waves per SIMD requested from the register allocator (1: no cap,
// 4: at most 128 VGPRs); both variants are built and the launch configuration picks one.
template <int D, int ST, int OCC>
__global__ __launch_bounds__(256, OCC) void k_stream_collide(SCArgs a) {
  using C = Codec<ST>;
  using S = typename C::S;
  using T = typename C::T;
  constexpr int Q = nq<D>();
  __shared__ uint32_t s_off[27];
  __shared__ double s_red[3][8];
  const int G = gridDim.x;
  const int me = (a.remap && (G & 7) == 0) ? xcd_perm(blockIdx.x, G) : blockIdx.x;
  for (int base = 0; base < a.n_items; base += G) {
    const int idx = base + me;
    if (idx >= a.n_items) break;
    const WorkItem w = a.items[idx];
    const LevelStatic &L = a.lev[w.level];
    __syncthreads();
    if (threadIdx.x < 27) {
      const int nb = L.nbr[(size_t)w.brick * 27 + threadIdx.x];
      s_off[threadIdx.x] = (uint32_t)(nb < 0 ? 0 : nb) * brick_bytes<D, ST>();
    }
    __syncthreads();
    const char *__restrict__ srcb = (const char *)a.src[w.level];
    S *__restrict__ dst = (S *)a.dst[w.level] + (size_t)w.brick * Q * BN;
    const T beta = T(L.beta);
    double fd[3] = {0, 0, 0};
    auto boff = [&](int code) { return s_off[code]; };
    for (int n = threadIdx.x; n < BN; n += blockDim.x) {
      const uint8_t cls = L.cls[(size_t)w.brick * BN + n];
      if ((cls & CLS_MODE) < w.thr) continue;
      int x, y, z;
      node_xyz<D>(n, x, y, z);
      const Lane<D> ln(x, y, z);
      T h[Q];
      uint32_t mask = 0;
      if (cls & (CLS_LINKS | CLS_INLET | CLS_OUTFLOW)) {
        mask = L.mask[(size_t)w.brick * BN + n];
        pull_special<D, ST>(srcb, boff, ln, n, cls, mask, L, h);
      } else {
        pull_plain<D, ST>(srcb, boff, ln, h);
      }
      T F[3];
      node_force<D, T>(L, w.brick, n, F);
      const bool hf = (F[0] != T(0)) || (F[1] != T(0)) || (F[2] != T(0));
      S *o = dst + n;
      const T g = kbc_collide<D, T>(h, beta, F, hf, [&](int i, T v) { C::st(o + i * BN, v, T(wgt<D>(i))); });
      if (L.gamma) L.gamma[(size_t)w.brick * BN + n] = (float)g;
      if (cls & CLS_DRAG) {
        // population i leaves towards x + c_i; that node is solid when population Q-1-i
        // bounced back: momentum exchange 2 c_i f'_i, from the values just stored
        for (int i = 0; i < Q; ++i) {
          if (!((mask >> (Q - 1 - i)) & 1u)) continue;
          const double fi = wgt<D>(i) + (double)C::ld(o + i * BN, T(wgt<D>(i)));
          fd[0] += 2.0 * (double)cxo(i) * fi;
          fd[1] += 2.0 * (double)cyo(i) * fi;
          fd[2] += 2.0 * (double)czo<D>(i) * fi;
        }
      }
    }
    if (w.drag) {  // deterministic block reduction of the momentum exchange
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
          L.drag[(size_t)w.brick * 3 + k] += s;
        }
      }
    }
  }
}

// ---------------------------------------------------------------- interface gather
// Post-stream (rho - 1, u, f^neq) at coarse-aligned interpolation points, parent
// values brought to child scale (Eq. f_neq_rescaling_iso); one staged row per point.
template <int D> __host__ __device__ constexpr int stage_width() { return D == 3 ? 32 : 12; }

template <int D, int ST> __global__ __launch_bounds__(256) void k_gather(GatherArgs a) {
  using C = Codec<ST>;
  using T = typename C::T;
  constexpr int Q = nq<D>();
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.n) return;
  const GPoint g = a.pts[p];
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
template <typename T> struct V4;
template <> struct V4<float> {
  typedef float type __attribute__((ext_vector_type(4)));
};
template <> struct V4<double> {
  typedef double type __attribute__((ext_vector_type(4)));
};

template <int D, int ST> __global__ __launch_bounds__(128) void k_couple(CoupleArgs a) {
  using C = Codec<ST>;
  using S = typename C::S;
  using T = typename C::T;
  using V = typename V4<T>::type;
  constexpr int Q = nq<D>();
  constexpr int SW = stage_width<D>();
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.n) return;
  const CItem c = a.items[t];
  const LevelStatic &L = a.lev[c.level];
  T h[Q];
  if (c.kind == 0) {
    T acc[SW];
#pragma unroll
    for (int v = 0; v < SW; ++v) acc[v] = 0;
    const T *stage = (const T *)a.stage;
    for (int e = c.a; e < c.a + c.b; ++e) {
      const StencilEntry s = a.sten[e];
      const T w = T(s.w);
      const V *row = (const V *)(stage + (size_t)s.slot * SW);
#pragma unroll
      for (int v = 0; v < SW / 4; ++v) {
        const V r = row[v];
        acc[4 * v + 0] = fma(w, r.x, acc[4 * v + 0]);
        acc[4 * v + 1] = fma(w, r.y, acc[4 * v + 1]);
        acc[4 * v + 2] = fma(w, r.z, acc[4 * v + 2]);
        acc[4 * v + 3] = fma(w, r.w, acc[4 * v + 3]);
      }
    }
    T u[3] = {acc[1], acc[2], D == 3 ? acc[3] : T(0)};
    T q[Q];
    eq_dev<D, T>(acc[0], u, q);
#pragma unroll
    for (int i = 0; i < Q; ++i) h[i] = acc[1 + D + i] + T(wgt<D>(i)) * q[i];
  } else {
    const int fl = c.level + 1;
    const LevelStatic &Lf = a.lev[fl];
    const char *srcb = (const char *)a.src[fl];
    const int32_t *nb = Lf.nbr + (size_t)c.a * 27;
    auto boff = [&](int code) { return (uint32_t)nb[code] * brick_bytes<D, ST>(); };
    int x, y, z;
    node_xyz<D>(c.b, x, y, z);
    const Lane<D> ln(x, y, z);
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
  }
  T F[3];
  node_force<D, T>(L, c.brick, c.node, F);
  const bool hf = (F[0] != T(0)) || (F[1] != T(0)) || (F[2] != T(0));
  S *o = (S *)a.dst[c.level] + (size_t)c.brick * Q * BN + c.node;
  const T g = kbc_collide<D, T>(h, T(L.beta), F, hf, [&](int i, T v) { C::st(o + i * BN, v, T(wgt<D>(i))); });
  if (L.gamma) L.gamma[(size_t)c.brick * BN + c.node] = (float)g;
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

int launch_stream_collide(int D, int st, const SCArgs &a, LaunchCfg cfg, void *stream) {
  if (a.n_items <= 0) return 0;
  const int grid = cfg.grid > 0 ? cfg.grid : a.n_items;
  const int thr = cfg.threads > 0 ? cfg.threads : 256;
  if (cfg.occ >= 4)
    ELBM_DISPATCH(D, st, (k_stream_collide<DD, SS, 4><<<grid, thr, 0, (hipStream_t)stream>>>(a)));
  else
    ELBM_DISPATCH(D, st, (k_stream_collide<DD, SS, 1><<<grid, thr, 0, (hipStream_t)stream>>>(a)));
  return ck();
}

int launch_gather(int D, int st, const GatherArgs &a, void *stream) {
  if (a.n <= 0) return 0;
  const int grid = (a.n + 255) / 256;
  ELBM_DISPATCH(D, st, (k_gather<DD, SS><<<grid, 256, 0, (hipStream_t)stream>>>(a)));
  return ck();
}

int launch_couple(int D, int st, const CoupleArgs &a, void *stream) {
  if (a.n <= 0) return 0;
  const int grid = (a.n + 127) / 128;
  ELBM_DISPATCH(D, st, (k_couple<DD, SS><<<grid, 128, 0, (hipStream_t)stream>>>(a)));
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

int stage_row_width(int D) { return D == 3 ? stage_width<3>() : stage_width<2>(); }

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
