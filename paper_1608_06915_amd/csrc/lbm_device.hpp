// lbm_device.hpp -- device building blocks shared by the forward and adjoint kernels:
// lattice constants, storage codecs, the equilibrium and KBC collision in shifted
// variables, and the pull addressing over bricks.
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
#pragma once
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
// Raw buffer resource over one level's population buffer: loads and stores address
// it with a per-lane 32-bit offset plus a wave-uniform scalar offset (no 64-bit
// address arithmetic per access); accesses past `bytes` read zero and are dropped.
typedef __amdgpu_buffer_rsrc_t Rsrc;
__device__ inline Rsrc buf_rsrc(const void *base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, (int)bytes, 0x00020000);
}

// Cache policy of the population stores through buffer resources.  FP64 and FP32:
// non-temporal (the NT bit of the gfx94x cache-policy operand) -- a stored population
// is read only by the next launch, so it streams past the L2 (measured: stream-collide
// 63 -> 60 us on the FP32 channel).  16-bit storage: default policy (non-temporal
// 2-byte stores measured slower).
constexpr int ST_POLICY = 2, ST_POLICY16 = 0;

template <int ST> struct Codec;
template <> struct Codec<ST_F64> {
  typedef double S;
  typedef double T;
  __device__ static inline T ld(const S *p, T w) { return *p - w; }
  __device__ static inline void st(S *p, T h, T w) { *p = w + h; }
  __device__ static inline T ldb(Rsrc r, uint32_t v, uint32_t s, T w) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, v, s, 0)) - w;
  }
  __device__ static inline S ldr(Rsrc r, uint32_t v, uint32_t s) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, v, s, 0));
  }
  __device__ static inline T dec(S x, T w) { return x - w; }
  __device__ static inline void stb(Rsrc r, uint32_t v, uint32_t s, T h, T w) {
    typedef decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0)) V2;
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, w + h), r, v, s, ST_POLICY);
  }
};
template <> struct Codec<ST_F32> {
  typedef float S;
  typedef float T;
  __device__ static inline T ld(const S *p, T w) { return *p - w; }
  __device__ static inline void st(S *p, T h, T w) { *p = w + h; }
  __device__ static inline T ldb(Rsrc r, uint32_t v, uint32_t s, T w) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, v, s, 0)) - w;
  }
  __device__ static inline S ldr(Rsrc r, uint32_t v, uint32_t s) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, v, s, 0));
  }
  __device__ static inline T dec(S x, T w) { return x - w; }
  __device__ static inline void stb(Rsrc r, uint32_t v, uint32_t s, T h, T w) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, w + h), r, v, s, ST_POLICY);
  }
};
template <> struct Codec<ST_F16S> {
  typedef uint16_t S;
  typedef float T;
  __device__ static inline T unpack(uint16_t b) { return __half2float(__ushort_as_half(b)); }
  __device__ static inline uint16_t pack(T h) { return __half_as_ushort(__float2half_rn(h)); }
  __device__ static inline T ld(const S *p, T) { return unpack(*p); }
  __device__ static inline void st(S *p, T h, T) { *p = pack(h); }
  __device__ static inline S ldr(Rsrc r, uint32_t v, uint32_t s) {
    return __builtin_amdgcn_raw_buffer_load_b16(r, v, s, 0);
  }
  __device__ static inline T dec(S x, T) { return unpack(x); }
  __device__ static inline T ldb(Rsrc r, uint32_t v, uint32_t s, T) {
    return unpack(__builtin_amdgcn_raw_buffer_load_b16(r, v, s, 0));
  }
  __device__ static inline void stb(Rsrc r, uint32_t v, uint32_t s, T h, T) {
    __builtin_amdgcn_raw_buffer_store_b16(pack(h), r, v, s, ST_POLICY16);
  }
};
template <> struct Codec<ST_BF16S> {
  typedef uint16_t S;
  typedef float T;
  __device__ static inline T unpack(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }
  __device__ static inline uint16_t pack(T h) {
    uint32_t b = __float_as_uint(h);
    if ((b & 0x7fffffffu) > 0x7f800000u) return (uint16_t)0x7fc0u;
    b += 0x7fffu + ((b >> 16) & 1u);  // round to nearest, ties to even
    return (uint16_t)(b >> 16);
  }
  __device__ static inline T ld(const S *p, T) { return unpack(*p); }
  __device__ static inline void st(S *p, T h, T) { *p = pack(h); }
  __device__ static inline S ldr(Rsrc r, uint32_t v, uint32_t s) {
    return __builtin_amdgcn_raw_buffer_load_b16(r, v, s, 0);
  }
  __device__ static inline T dec(S x, T) { return unpack(x); }
  __device__ static inline T ldb(Rsrc r, uint32_t v, uint32_t s, T) {
    return unpack(__builtin_amdgcn_raw_buffer_load_b16(r, v, s, 0));
  }
  __device__ static inline void stb(Rsrc r, uint32_t v, uint32_t s, T h, T) {
    __builtin_amdgcn_raw_buffer_store_b16(pack(h), r, v, s, ST_POLICY16);
  }
};

template <int D, int ST> __device__ constexpr uint32_t brick_bytes() {
  return (uint32_t)(nq<D>() * BN * sizeof(typename Codec<ST>::S));
}

// FP32 uses the hardware reciprocal and square root (about 1 ulp); FP64 keeps IEEE
// division and square root.
__device__ inline float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double rcp(double x) { return 1.0 / x; }
__device__ inline float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ inline double sqrt_(double x) { return sqrt(x); }

// ---------------------------------------------------------------- balanced sums
// Sums over the populations are balanced trees over the contributing populations
// only (selected at compile time), so the dependency chains are log2 deep instead
// of Q long (instruction-level parallelism per wave).
enum {
  P_ALL, P_XP, P_XN, P_YP, P_YN, P_ZP, P_ZN,  // sign of one velocity component
  P_XZP, P_XZN, P_YZP, P_YZN, P_XYP,          // c_a^2 - c_b^2 = +-1, 2-D c_x^2 - c_y^2
  P_XYN, P_MXYP, P_MXYN, P_MXZP, P_MXZN,      // 2-D c_x^2 - c_y^2 = -1; c_a c_b = +-1
  P_MYZP, P_MYZN, P_SHEAR                     // c_y c_z = +-1; shear part nonzero
};
template <int D, int P> __host__ __device__ constexpr bool pick(int i) {
  const int x = cxo(i), y = cyo(i), z = czo<D>(i);
  switch (P) {
    case P_ALL: return true;
    case P_XP: return x == 1;
    case P_XN: return x == -1;
    case P_YP: return y == 1;
    case P_YN: return y == -1;
    case P_ZP: return z == 1;
    case P_ZN: return z == -1;
    case P_XZP: return x * x - z * z == 1;
    case P_XZN: return x * x - z * z == -1;
    case P_YZP: return y * y - z * z == 1;
    case P_YZN: return y * y - z * z == -1;
    case P_XYP: return x * x - y * y == 1;
    case P_XYN: return x * x - y * y == -1;
    case P_MXYP: return x * y == 1;
    case P_MXYN: return x * y == -1;
    case P_MXZP: return x * z == 1;
    case P_MXZN: return x * z == -1;
    case P_MYZP: return y * z == 1;
    case P_MYZN: return y * z == -1;
    case P_SHEAR: return x * x + y * y + z * z == 1 || x * x + y * y + z * z == 2;
  }
  return false;
}
template <int D, int P> __host__ __device__ constexpr int npick(int lo, int n) {
  int c = 0;
  for (int i = lo; i < lo + n; ++i) c += pick<D, P>(i) ? 1 : 0;
  return c;
}
// sum of f(i) over i in [LO, LO+N) with pick<D,P>(i); the range has >= 1 term
template <int D, int P, int LO, int N, typename T, typename F> __device__ inline T tsel(F f) {
  if constexpr (N == 1) {
    return f(LO);
  } else {
    constexpr int NL = N / 2;
    constexpr int cl = npick<D, P>(LO, NL), cr = npick<D, P>(LO + NL, N - NL);
    if constexpr (cl == 0) return tsel<D, P, LO + NL, N - NL, T>(f);
    else if constexpr (cr == 0) return tsel<D, P, LO, NL, T>(f);
    else return tsel<D, P, LO, NL, T>(f) + tsel<D, P, LO + NL, N - NL, T>(f);
  }
}
template <int D, int P, typename T, typename F> __device__ inline T tsum(F f) {
  return tsel<D, P, 0, nq<D>(), T>(f);
}

template <int I> struct Ic {
  static constexpr int value = I;
};
// compile-time loop: f(Ic<I>) for I in [B, E); indices are constants before any
// optimisation pass, so small arrays indexed by them stay in registers
template <int B, int E, typename F> __device__ inline void static_for(F &&f) {
  if constexpr (B < E) {
    f(Ic<B>());
    static_for<B + 1, E>(f);
  }
}

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
  auto v = [&](int i) { return h[i]; };
  drho = tsum<D, P_ALL, T>(v);
  j[0] = tsum<D, P_XP, T>(v) - tsum<D, P_XN, T>(v);
  j[1] = tsum<D, P_YP, T>(v) - tsum<D, P_YN, T>(v);
  j[2] = D == 3 ? tsum<D, P_ZP, T>(v) - tsum<D, P_ZN, T>(v) : T(0);
}

// Density, momentum and second moments of h by an axis cascade (sums over c_z, then
// c_y, then c_x, keeping the orders needed): drho = sum h, j = sum c h,
// m2 = {sum c_x^2 h, sum c_y^2 h, sum c_z^2 h, sum c_x c_y h, sum c_x c_z h, sum c_y c_z h}.
template <int D, typename T>
__device__ inline void hmoments(const T (&h)[nq<D>()], T &drho, T (&j)[3], T (&m2)[6]) {
  T H[3][3][3];  // h by velocity (c_x + 1, c_y + 1, c_z + 1)
  static_for<0, nq<D>()>([&](auto I) {
    constexpr int i = decltype(I)::value;
    H[cxo(i) + 1][cyo(i) + 1][czo<D>(i) + 1] = h[i];
  });
  // per x: sums over y of the z-moments 0, 1, 2 (0 and 1 also with weight c_y, 0 with c_y^2)
  T t0[3], ty[3], tyy[3], z1[3], z1y[3], z2[3];
#pragma unroll
  for (int x = 0; x < 3; ++x) {
    T s0[3], s1[3], s2[3];  // by y: sum_z h, sum_z c_z h, sum_z c_z^2 h
#pragma unroll
    for (int y = 0; y < 3; ++y) {
      if (D == 3) {
        s2[y] = H[x][y][2] + H[x][y][0];
        s1[y] = H[x][y][2] - H[x][y][0];
        s0[y] = s2[y] + H[x][y][1];
      } else {
        s0[y] = H[x][y][1];
        s1[y] = s2[y] = T(0);
      }
    }
    tyy[x] = s0[2] + s0[0];
    ty[x] = s0[2] - s0[0];
    t0[x] = tyy[x] + s0[1];
    z1[x] = (s1[2] + s1[0]) + s1[1];
    z1y[x] = s1[2] - s1[0];
    z2[x] = (s2[2] + s2[0]) + s2[1];
  }
  const T c0 = t0[2] + t0[0];
  drho = c0 + t0[1];
  j[0] = t0[2] - t0[0];
  j[1] = (ty[2] + ty[0]) + ty[1];
  j[2] = (z1[2] + z1[0]) + z1[1];
  m2[0] = c0;
  m2[1] = (tyy[2] + tyy[0]) + tyy[1];
  m2[2] = (z2[2] + z2[0]) + z2[1];
  m2[3] = ty[2] - ty[0];
  m2[4] = z1[2] - z1[0];
  m2[5] = (z1y[2] + z1y[0]) + z1y[1];
}

// ---------------------------------------------------------------- KBC collision
// Post-collision h' = h - beta (2 ds + gamma dh) (Eq. f_equations with Eq. f_mirr),
// gamma from Eq. gamma_min_approx, plus the exact-difference forcing of Sec. III.A.
// h is overwritten by the deviation d = h - (f^eq - W); the post-collision value of
// population i is handed to st(i, h'_i).  F: force density in level units.
template <int D, typename T, typename Store>
__device__ inline T kbc_collide(T (&h)[nq<D>()], T beta, const T F[3], bool has_force, Store st) {
  constexpr int Q = nq<D>();
  T drho, j[3], m2[6];
  hmoments<D, T>(h, drho, j, m2);
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
  // deviatoric second moments of d = f - f^eq: those of h less those of the product
  // equilibrium, which are exact: sum_i W_i q_i c_a^2 = (1 + drho)(1/3 + 2 sig_a / 3) - 1/3
  // and sum_i W_i q_i c_a c_b = (1 + drho) u_a u_b = j_a u_b, with sig_a = -a[a][1] the
  // axis factor's sigma (the 1/3 of the lattice weights cancels in the differences)
  const T r23 = (T(1) + drho) * T(2.0 / 3.0);
  T N1, N2 = 0, Pxz = 0, Pyz = 0;
  if constexpr (D == 2) {
    N1 = fma(-r23, a[1][1] - a[0][1], m2[0] - m2[1]);
  } else {
    N1 = fma(-r23, a[2][1] - a[0][1], m2[0] - m2[2]);
    N2 = fma(-r23, a[2][1] - a[1][1], m2[1] - m2[2]);
    Pxz = fma(-j[0], u[2], m2[4]);
    Pyz = fma(-j[1], u[2], m2[5]);
  }
  const T Pxy = fma(-j[0], u[1], m2[3]);
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
  // entropic scalar products <ds|dh>, <dh|dh> with weight 1/f^eq_i.  The lattice
  // weights are products of the 1-D weights w(0) = 2/3, w(+-1) = 1/6, so
  // 1/f^eq_i = ir * prod_a 1/(w(c_a) (1 + a_a(c_a))): one reciprocal per axis and
  // velocity component.  The sums run as three fused multiply-add chains, one per
  // velocity component of the last axis (c_z; c_y in 2-D), whose factor 1/(w (1 + a))
  // -- with the density folded in -- multiplies each chain's sum once at the end.
  T A = 0, B = 0;
  {
    T r0[3], r1[3], rl[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const T w = k == 1 ? T(2.0 / 3.0) : T(1.0 / 6.0);
      r0[k] = rcp(fma(w, a[0][k], w));
      if (D == 3) {
        r1[k] = rcp(fma(w, a[1][k], w));
        rl[k] = ir * rcp(fma(w, a[2][k], w));
      } else {
        r1[k] = T(1);
        rl[k] = ir * rcp(fma(w, a[1][k], w));
      }
    }
    T rxy[9];
#pragma unroll
    for (int cy = 0; cy < 3; ++cy)
#pragma unroll
      for (int cx = 0; cx < 3; ++cx) rxy[cx + 3 * cy] = D == 3 ? r0[cx] * r1[cy] : r0[cx];
    T Ap[3] = {0, 0, 0}, Bp[3] = {0, 0, 0};
    static_for<0, Q>([&](auto I) {
      constexpr int i = decltype(I)::value;
      constexpr int cx = cxo(i), cy = cyo(i), cz = czo<D>(i);
      constexpr int lane = D == 3 ? cz + 1 : cy + 1;
      const T ifq = rxy[(cx + 1) + 3 * (cy + 1)];  // 1/f^eq_i without the last axis' factor
      const T ds = dsv(i);
      const T dh = h[i] - ds;
      const T t = dh * ifq;
      Bp[lane] = fma(t, dh, Bp[lane]);
      if constexpr (cx * cx + cy * cy + cz * cz == 1 || cx * cx + cy * cy + cz * cz == 2)
        Ap[lane] = fma(t, ds, Ap[lane]);  // the shear part ds is nonzero
    });
    A = fma(rl[2], Ap[2], fma(rl[1], Ap[1], rl[0] * Ap[0]));
    B = fma(rl[2], Bp[2], fma(rl[1], Bp[1], rl[0] * Bp[0]));
  }
  const T ib = rcp(beta);
  T gamma = T(2);
  if (B > T(0)) {
    const T g = ib - (T(2) - ib) * (A * rcp(B));
    if (isfinite(g)) gamma = g;
  }
  // h' = W q' + d - 2 beta ds - beta gamma (d - ds) = W q' + c1 d + c2 ds, with c2 ds
  // taking six distinct values (q' the equilibrium of the forced velocity, if any)
  // (each written so that only one evaluation is possible: contraction of a product into
  // a sum is up to the compiler, and every instance of this function must round alike)
  const T c1 = fma(-beta, gamma, T(1)), c2 = beta * (gamma - T(2));
  const T c2sX = c2 * sX, c2sY = c2 * sY, c2sZ = c2 * sZ, c2pxy = c2 * pxy, c2pxz = c2 * pxz, c2pyz = c2 * pyz;
  auto c2ds = [&](int i) -> T {
    const int x = cxo(i), y = cyo(i), z = czo<D>(i);
    const int nz = x * x + y * y + z * z;
    if (nz == 1) return x ? c2sX : (y ? c2sY : c2sZ);
    if (nz == 2) return (z == 0) ? T(x * y) * c2pxy : ((y == 0) ? T(x * z) * c2pxz : T(y * z) * c2pyz);
    return T(0);
  };
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
    for (int i = 0; i < Q; ++i) st(i, fma(c1, h[i], fma(T(wgt<D>(i)), q_of<D>(qxy2, a2, i), c2ds(i))));
  } else {
#pragma unroll
    for (int i = 0; i < Q; ++i) st(i, fma(c1, h[i], fma(T(wgt<D>(i)), q_of<D>(qxy, a, i), c2ds(i))));
  }
  return gamma;
}

// Tables that no kernel writes are read through the constant address space: with a
// wave-uniform address that is a scalar load into SGPRs instead of a vector load
// followed by readfirstlane.
template <typename T> using cptr = const __attribute__((address_space(4))) T *;
template <typename T> __device__ inline cptr<T> cst(const T *p) { return (cptr<T>)p; }

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

template <int D> struct BulkLane {
  bool xlo, xhi, ylo, yhi;  // per lane: on the low/high x (y) face of the brick
  uint32_t mxlo, mxhi, mylo, myhi;  // the same as all-ones / zero masks
  int lx[3], ly[3];         // local x, y of the source for c = +1, 0, -1 (index 1 - c)
  int lz[3];                // local z part (uniform)
  bool zlo, zhi;            // uniform
  __device__ inline BulkLane(int x, int y, int z) {
    using Bk = Brick<D>;
    xlo = x == 0;
    xhi = x == Bk::BX - 1;
    ylo = y == 0;
    yhi = y == Bk::BY - 1;
    mxlo = 0u - (uint32_t)xlo;
    mxhi = 0u - (uint32_t)xhi;
    mylo = 0u - (uint32_t)ylo;
    myhi = 0u - (uint32_t)yhi;
    static_for<0, 3>([&](auto K) {
      constexpr int k = decltype(K)::value;
      lx[k] = (x - 1 + k) & (Bk::BX - 1);
      ly[k] = Bk::BX * ((y - 1 + k) & (Bk::BY - 1));
      lz[k] = D == 3 ? Bk::BX * Bk::BY * ((z - 1 + k) & (Bk::BZ - 1)) : 0;
    });
    zlo = D == 3 && z == 0;
    zhi = D == 3 && z == Bk::BZ - 1;
  }
};

// Bulk pull.  mid[k]: byte offset of the neighbour brick at displacement code 9 + k
// (same z-layer of bricks), side[k]: the brick layer below (z on the low brick face)
// or above (z on the high face) -- z is uniform over a wavefront, so one side layer
// suffices.  Offsets are wave-uniform scalars.  A lane on an x (y) brick face takes
// the neighbour brick for that axis; the choice is formed branch-free as
//   base = O + (mx & dX) + (my & dY) + (mx & my & dXY)
// with the lane's face masks and scalar differences of the candidate offsets (a
// select between two scalars is not one vector instruction here, and as a select it
// compiles to divergent branches).
template <int D, int I>
__device__ inline uint32_t bulk_base(const uint32_t (&mid)[9], const uint32_t (&side)[9], const BulkLane<D> &b) {
  constexpr int cx = cxo(I), cy = cyo(I), cz = czo<D>(I);
  // candidate brick offsets (wave-uniform): x index kx, y index ky into the 3x3 layer;
  // interior lanes use (1, 1)
  auto U = [&](int kx, int ky) -> uint32_t {
    const int k = kx + 3 * ky;
    uint32_t v = mid[k];
    if constexpr (cz == 1) v = b.zlo ? side[k] : mid[k];
    if constexpr (cz == -1) v = b.zhi ? side[k] : mid[k];
    return __builtin_amdgcn_readfirstlane(v);
  };
  constexpr int ex = cx == 1 ? 0 : 2, ey = cy == 1 ? 0 : 2;  // edge candidates
  const uint32_t o11 = U(1, 1);
  uint32_t base = o11;
  if constexpr (cx != 0) {
    const uint32_t mx = cx == 1 ? b.mxlo : b.mxhi;
    base += mx & (U(ex, 1) - o11);
    if constexpr (cy != 0) {
      const uint32_t my = cy == 1 ? b.mylo : b.myhi;
      base += my & (U(1, ey) - o11);
      base += (mx & my) & (U(ex, ey) - U(ex, 1) - U(1, ey) + o11);
    }
  } else if constexpr (cy != 0) {
    const uint32_t my = cy == 1 ? b.mylo : b.myhi;
    base += my & (U(1, ey) - o11);
  }
  return base;
}

template <int D, int ST, typename LD>
__device__ inline void pull_bulk_with(const uint32_t (&mid)[9], const uint32_t (&side)[9], const BulkLane<D> &b,
                                      LD ld) {
  using S = typename Codec<ST>::S;
  static_for<0, nq<D>()>([&](auto I) {
    constexpr int i = decltype(I)::value;
    constexpr int cx = cxo(i), cy = cyo(i), cz = czo<D>(i);
    const uint32_t base = bulk_base<D, i>(mid, side, b);
    const int loc = b.lx[1 - cx] + b.ly[1 - cy] + b.lz[1 - cz];
    ld(i, base + (uint32_t)(loc * (int)sizeof(S)), (uint32_t)(i * BN * (int)sizeof(S)));
  });
}

template <int D, int ST>
__device__ inline void pull_bulk(Rsrc src, const uint32_t (&mid)[9], const uint32_t (&side)[9],
                                 const BulkLane<D> &b, typename Codec<ST>::T (&h)[nq<D>()]) {
  using C = Codec<ST>;
  using T = typename C::T;
  pull_bulk_with<D, ST>(mid, side, b, [&](int i, uint32_t v, uint32_t s) { h[i] = C::ldb(src, v, s, T(wgt<D>(i))); });
}

// Pull of a node with special links (mask bit i set): bounce-back (CLS_LINKS) reads
// the node's own population Q-1-i, an outflow link (CLS_OUTFLOW) reads population i one
// node upstream of x - c_i (shift oshift back into the domain), an inlet link
// (CLS_INLET) takes the inlet value.  The other links use the bulk addressing.  Every
// address is formed with selects and every load is issued, so a wavefront keeps all
// of its loads in flight.  nbo(code): byte offset of the neighbour brick of a
// displacement code (an LDS table); own: byte offset of the node's brick; Lc: the
// level's constants (scalar loads).
template <int D, int ST, typename NBO, typename LD>
__device__ inline void pull_links_with(const uint32_t (&md)[9], const uint32_t (&sd)[9], const BulkLane<D> &b,
                                       NBO nbo, uint32_t own, int x, int y, int z, int n, uint32_t cls,
                                       uint32_t mask, cptr<LevelStatic> Lc, LD ld) {
  using S = typename Codec<ST>::S;
  using Bk = Brick<D>;
  constexpr int Q = nq<D>();
  const bool bb = (cls & CLS_LINKS) != 0, ofl = (cls & CLS_OUTFLOW) != 0;
  uint32_t ov[Q];
  const bool any_ofl = __builtin_amdgcn_ballot_w64(ofl) != 0;  // wave-uniform
  if (any_ofl) {
    const int ox = Lc->oshift[0], oy = Lc->oshift[1], oz = Lc->oshift[2];
    static_for<0, Q>([&](auto I) {
      constexpr int i = decltype(I)::value;
      const int sx = x - cxo(i) - ox, sy = y - cyo(i) - oy, sz = z - czo<D>(i) - oz;
      const int code = side<Bk::BX>(sx) + 3 * side<Bk::BY>(sy) + 9 * (D == 3 ? side<Bk::BZ>(sz) : 1);
      const int loc = (sx & (Bk::BX - 1)) + Bk::BX * ((sy & (Bk::BY - 1)) + Bk::BY * (D == 3 ? (sz & (Bk::BZ - 1)) : 0));
      ov[i] = nbo(code) + (uint32_t)((i * BN + loc) * (int)sizeof(S));
    });
  }
  static_for<0, Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    constexpr int cx = cxo(i), cy = cyo(i), cz = czo<D>(i);
    const uint32_t base = bulk_base<D, i>(md, sd, b);
    const int loc = b.lx[1 - cx] + b.ly[1 - cy] + b.lz[1 - cz];
    const bool hit = (mask >> i) & 1u;
    uint32_t v = base + (uint32_t)((i * BN + loc) * (int)sizeof(S));
    v = (bb && hit) ? own + (uint32_t)(((Q - 1 - i) * BN + n) * (int)sizeof(S)) : v;
    if (any_ofl) v = (ofl && hit) ? ov[i] : v;
    // the weights are symmetric (W_i = W_{Q-1-i}): one shift for every source
    ld(i, v, 0u);
  });
}

// inlet links take the inlet populations (after the loads of pull_links_with)
template <int D, typename T>
__device__ inline void apply_inlet(uint32_t cls, uint32_t mask, cptr<LevelStatic> Lc, T (&h)[nq<D>()]) {
  if (cls & CLS_INLET) {
    static_for<0, nq<D>()>([&](auto I) {
      constexpr int i = decltype(I)::value;
      const T hv = T(Lc->hin[i]);
      if ((mask >> i) & 1u) h[i] = hv;
    });
  }
}

template <int D, int ST, typename NBO>
__device__ inline void pull_links(Rsrc src, const uint32_t (&md)[9], const uint32_t (&sd)[9], const BulkLane<D> &b,
                                  NBO nbo, uint32_t own, int x, int y, int z, int n, uint32_t cls, uint32_t mask,
                                  cptr<LevelStatic> Lc, typename Codec<ST>::T (&h)[nq<D>()]) {
  using C = Codec<ST>;
  using T = typename C::T;
  pull_links_with<D, ST>(md, sd, b, nbo, own, x, y, z, n, cls, mask, Lc,
                         [&](int i, uint32_t v, uint32_t s) { h[i] = C::ldb(src, v, s, T(wgt<D>(i))); });
  apply_inlet<D, T>(cls, mask, Lc, h);
}

// neighbour-brick byte offsets of the bulk pull; nbp(k): neighbour brick of
// displacement code k (missing -> 0)
template <int D, int ST, typename NB>
__device__ inline void bulk_offsets(NB nbp, int z, uint32_t (&mid)[9], uint32_t (&side)[9]) {
  using Bk = Brick<D>;
  const int sl = (D == 3 && z == 0) ? 0 : ((D == 3 && z == Bk::BZ - 1) ? 18 : 9);
  static_for<0, 9>([&](auto K) {
    constexpr int k = decltype(K)::value;
    const int m = nbp(9 + k);
    const int s = nbp(sl + k);
    mid[k] = (uint32_t)(m < 0 ? 0 : m) * brick_bytes<D, ST>();
    side[k] = (uint32_t)(s < 0 ? 0 : s) * brick_bytes<D, ST>();
  });
}

template <int D> __device__ inline void node_xyz(int n, int &x, int &y, int &z) {
  using Bk = Brick<D>;
  x = n & (Bk::BX - 1);
  y = (n >> Bk::LX) & (Bk::BY - 1);
  z = D == 3 ? (n >> (Bk::LX + Bk::LY)) : 0;
}

// Item of workgroup b in a grid of G.  The hardware deals workgroups round-robin to
// the 8 XCDs (b & 7), each with its own L2.  mode 0 (and 1, whose mapping is a table
// built on the host): identity; mode B >= 2: runs of B consecutive items go to one XCD
// and the runs are dealt round-robin, so bricks that share halo lines (consecutive
// bricks are x-neighbours) meet in one L2 while every XCD still sweeps the whole item
// range; workgroups past the last whole round of 8 runs keep their own index.  Every
// mode is a bijection of [0, G).
__device__ inline int xcd_item(int b, int G, int mode) {
  if (mode >= 2) {
    const int round = 8 * mode;
    if (b < G / round * round) {
      const int l = b >> 3;  // position of b among its XCD's workgroups
      return ((l / mode) * 8 + (b & 7)) * mode + l % mode;
    }
  }
  return b;
}


template <int D> __host__ __device__ constexpr int stage_width() { return D == 3 ? 32 : 12; }
// row stride of staged rows in LDS: a row that is a multiple of 128 bytes (all banks)
// gets one vector (4 elements) of padding, so that the rows that different lanes read
// start in different bank groups; rows are copied and read as 4-element vectors
template <int D, typename T> __host__ __device__ constexpr int lds_stride() {
  return (stage_width<D>() * (int)sizeof(T)) % 128 == 0 ? stage_width<D>() + 4 : stage_width<D>();
}
static_assert(lds_stride<3, float>() % 4 == 0 && lds_stride<3, double>() % 4 == 0 &&
                  lds_stride<2, float>() % 4 == 0 && lds_stride<2, double>() % 4 == 0,
              "staged rows are accessed as 4-element vectors");

template <typename T> struct V4;
template <> struct V4<float> {
  typedef float type __attribute__((ext_vector_type(4)));
};
template <> struct V4<double> {
  typedef double type __attribute__((ext_vector_type(4)));
};


}  // namespace elbm
