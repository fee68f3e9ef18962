// Shared device/host definitions of the DD-alpha-AMG library (gfx950).
//
// Fine-lattice device layout ("block layout"): the lattice (T,Z,Y,X) is cut
// into blocks of b = (bT,bZ,bY,bX) sites, all extents even.  The block is the
// SAP domain and the first aggregate.  Blocks are numbered lexicographically
// over block coordinates (T slowest).  Inside a block the bs = bT*bZ*bY*bX
// sites are stored parity-major: slot = parity*half + (lexicographic local
// index >> 1), parity = (t+z+y+x) mod 2 (block origins are even, so local and
// global parity agree).  A field with C complex components per site is stored
// tiled inside each block (see fidx below).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <type_traits>

namespace ddamg {

template <class T>
struct alignas(2 * sizeof(T)) cx {
  T re, im;
};

template <class T> __host__ __device__ __forceinline__ cx<T> mk(T r, T i) { cx<T> z; z.re = r; z.im = i; return z; }
template <class T> __host__ __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return mk(a.re + b.re, a.im + b.im); }
template <class T> __host__ __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return mk(a.re - b.re, a.im - b.im); }
template <class T> __host__ __device__ __forceinline__ cx<T> operator-(cx<T> a) { return mk(-a.re, -a.im); }
template <class T> __host__ __device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
  return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <class T> __host__ __device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return mk(s * a.re, s * a.im); }
template <class T> __host__ __device__ __forceinline__ cx<T>& operator+=(cx<T>& a, cx<T> b) { a.re += b.re; a.im += b.im; return a; }
template <class T> __host__ __device__ __forceinline__ cx<T>& operator-=(cx<T>& a, cx<T> b) { a.re -= b.re; a.im -= b.im; return a; }
template <class T> __host__ __device__ __forceinline__ cx<T> conj(cx<T> a) { return mk(a.re, -a.im); }
template <class T> __host__ __device__ __forceinline__ cx<T> times_i(cx<T> a) { return mk(-a.im, a.re); }
template <class T> __host__ __device__ __forceinline__ cx<T> times_mi(cx<T> a) { return mk(a.im, -a.re); }
// a += b*c  and  a += conj(b)*c.  In FP32 on the device as two chained fused
// multiply-adds per component (the arithmetic-bound FP32 kernels: one
// instruction fewer per component than a product, a difference and a sum); in
// FP64 as sums of products (the FP64 kernels are bound by memory, and the
// shorter dependency chains keep their registers within budget).
template <class T> __host__ __device__ __forceinline__ void cmac(cx<T>& a, cx<T> b, cx<T> c) {
#ifdef __HIP_DEVICE_COMPILE__
  if constexpr (std::is_same<T, float>::value) {
    a.re = __builtin_fmaf(-b.im, c.im, __builtin_fmaf(b.re, c.re, a.re));
    a.im = __builtin_fmaf(b.im, c.re, __builtin_fmaf(b.re, c.im, a.im));
    return;
  }
#endif
  a.re += b.re * c.re - b.im * c.im;
  a.im += b.re * c.im + b.im * c.re;
}
template <class T> __host__ __device__ __forceinline__ void cjmac(cx<T>& a, cx<T> b, cx<T> c) {
#ifdef __HIP_DEVICE_COMPILE__
  if constexpr (std::is_same<T, float>::value) {
    a.re = __builtin_fmaf(b.im, c.im, __builtin_fmaf(b.re, c.re, a.re));
    a.im = __builtin_fmaf(-b.im, c.re, __builtin_fmaf(b.re, c.im, a.im));
    return;
  }
#endif
  a.re += b.re * c.re + b.im * c.im;
  a.im += b.re * c.im - b.im * c.re;
}
template <class T> __host__ __device__ __forceinline__ T norm2(cx<T> a) { return a.re * a.re + a.im * a.im; }

// ---- storage types: complex numbers in double, float, fp16 or bf16 ----------
// 16-bit storage uses the compiler's native _Float16 and __bf16 types; every
// narrowing conversion rounds to nearest even.
using f16 = _Float16;
using bf16 = __bf16;
struct alignas(4) h2 { f16 re, im; };
struct alignas(4) b2 { bf16 re, im; };

template <class S> struct store_traits;
template <> struct store_traits<double> { using elem = cx<double>; };
template <> struct store_traits<float> { using elem = cx<float>; };
template <> struct store_traits<f16> { using elem = h2; };
template <> struct store_traits<bf16> { using elem = b2; };

template <class R, class S>
__device__ __forceinline__ cx<R> ld(const typename store_traits<S>::elem* p, long i);
template <> __device__ __forceinline__ cx<double> ld<double, double>(const cx<double>* p, long i) { return p[i]; }
template <> __device__ __forceinline__ cx<float> ld<float, float>(const cx<float>* p, long i) { return p[i]; }
template <> __device__ __forceinline__ cx<double> ld<double, float>(const cx<float>* p, long i) {
  cx<float> v = p[i]; return mk<double>(v.re, v.im);
}
template <> __device__ __forceinline__ cx<float> ld<float, double>(const cx<double>* p, long i) {
  cx<double> v = p[i]; return mk<float>((float)v.re, (float)v.im);
}
template <> __device__ __forceinline__ cx<float> ld<float, f16>(const h2* p, long i) {
  h2 v = p[i]; return mk<float>((float)v.re, (float)v.im);
}
template <> __device__ __forceinline__ cx<float> ld<float, bf16>(const b2* p, long i) {
  b2 v = p[i]; return mk<float>((float)v.re, (float)v.im);
}

template <class S, class R> __device__ __forceinline__ typename store_traits<S>::elem st_cvt(cx<R> v);
template <> __device__ __forceinline__ cx<double> st_cvt<double, double>(cx<double> v) { return v; }
template <> __device__ __forceinline__ cx<float> st_cvt<float, double>(cx<double> v) { return mk<float>((float)v.re, (float)v.im); }
template <> __device__ __forceinline__ cx<float> st_cvt<float, float>(cx<float> v) { return v; }
template <> __device__ __forceinline__ cx<double> st_cvt<double, float>(cx<float> v) { return mk<double>(v.re, v.im); }
template <> __device__ __forceinline__ h2 st_cvt<f16, double>(cx<double> v) {
  h2 r; r.re = (f16)v.re; r.im = (f16)v.im; return r;
}
template <> __device__ __forceinline__ b2 st_cvt<bf16, double>(cx<double> v) {
  b2 r; r.re = (bf16)v.re; r.im = (bf16)v.im; return r;
}

// ---- fine-lattice geometry -------------------------------------------------
// Inside a block, sites are grouped in tiles of TILE consecutive slots and a
// field is stored tile by tile, component-major inside a tile: component c of
// slot s of block B (field with C components) sits at
//   ((B * bs/TILE + s/TILE) * C + c) * TILE + s % TILE.
// A wavefront reading one component of 64 consecutive slots reads 64/TILE
// contiguous segments of TILE elements (FP64: 128 B, one cache line each),
// and the components of one site are a compile-time stride apart, so one
// address plus immediate offsets serves a whole site.
constexpr int TILE = 8;

// Twisted mass of the fine site terms: e on the even sites, o on the odd ones
// (the same value on both unless the operator carries a different twist on
// each parity).  TwistR is its copy in a kernel's arithmetic.
struct Twist {
  double e = 0, o = 0;
  Twist() = default;
  Twist(double t) : e(t), o(t) {}
  Twist(double te, double to) : e(te), o(to) {}
  Twist operator-() const { return Twist(-e, -o); }
  double mean() const { return 0.5 * (e + o); }
  double half_diff() const { return 0.5 * (o - e); }
};
template <class R>
struct TwistR {
  R e, o;
  TwistR() = default;
  __host__ __device__ TwistR(R te, R to) : e(te), o(to) {}
  __host__ explicit TwistR(const Twist& t) : e((R)t.e), o((R)t.o) {}
};

struct Geom {
  int L[4];      // extents T,Z,Y,X
  int b[4];      // block extents
  int nb[4];     // blocks per direction
  int nblocks;   // number of blocks
  int bs;        // sites per block
  int half;      // bs/2
  long V;        // sites
  int ndir;      // 4 (kept as data so loops over directions stay rolled)
};

// local coordinates of a slot
__host__ __device__ __forceinline__ void slot_local(const Geom& g, int s, int l[4]) {
  int p = s >= g.half ? 1 : 0;
  int idx = s - p * g.half;
  int bx2 = g.b[3] >> 1;
  int lx2 = idx % bx2;
  int r = idx / bx2;
  l[2] = r % g.b[2];
  r /= g.b[2];
  l[1] = r % g.b[1];
  l[0] = r / g.b[1];
  l[3] = 2 * lx2 + ((p + l[0] + l[1] + l[2]) & 1);
}

__host__ __device__ __forceinline__ int local_slot(const Geom& g, const int l[4]) {
  int p = (l[0] + l[1] + l[2] + l[3]) & 1;
  int idx = ((l[0] * g.b[1] + l[1]) * g.b[2] + l[2]) * (g.b[3] >> 1) + (l[3] >> 1);
  return p * g.half + idx;
}

__host__ __device__ __forceinline__ void block_coords(const Geom& g, int B, int c[4]) {
  c[3] = B % g.nb[3];
  int r = B / g.nb[3];
  c[2] = r % g.nb[2];
  r /= g.nb[2];
  c[1] = r % g.nb[1];
  c[0] = r / g.nb[1];
}

__host__ __device__ __forceinline__ int block_index(const Geom& g, const int c[4]) {
  return ((c[0] * g.nb[1] + c[1]) * g.nb[2] + c[2]) * g.nb[3] + c[3];
}

// global coordinates of (block, slot)
__host__ __device__ __forceinline__ void site_coords(const Geom& g, int B, int s, int x[4]) {
  int bc[4], l[4];
  block_coords(g, B, bc);
  slot_local(g, s, l);
  for (int d = 0; d < 4; ++d) x[d] = bc[d] * g.b[d] + l[d];
}

// (block, slot) of global coordinates
__host__ __device__ __forceinline__ void coords_site(const Geom& g, const int x[4], int& B, int& s) {
  int bc[4], l[4];
  for (int d = 0; d < 4; ++d) {
    bc[d] = x[d] / g.b[d];
    l[d] = x[d] - bc[d] * g.b[d];
  }
  B = block_index(g, bc);
  s = local_slot(g, l);
}

// neighbour of (B,s) one step in direction mu with sign dir (+1 / -1), periodic
__host__ __device__ __forceinline__ void neighbour(const Geom& g, int B, int s, int mu, int dir, int& Bn, int& sn) {
  int x[4];
  site_coords(g, B, s, x);
  x[mu] += dir;
  if (x[mu] == g.L[mu]) x[mu] = 0;
  if (x[mu] < 0) x[mu] = g.L[mu] - 1;
  coords_site(g, x, Bn, sn);
}

// Workgroups of a launch are dispatched round-robin over the 8 XCDs, each with
// its own L2.  Map workgroup w of nwg to a logical index so that every XCD
// owns one contiguous range of logical indices (lattice blocks that are
// neighbours in the block order then share an L2).  A bijection of [0, nwg).
__host__ __device__ __forceinline__ int xcd_remap(int w, int nwg) {
  int q = nwg >> 3, r = nwg & 7, x = w & 7, k = w >> 3;
  return x * q + (x < r ? x : r) + k;
}

// Workgroup -> lattice block for whole-lattice stencils.  The dispatcher
// hands workgroup w to XCD w % 8; here each group of m consecutive blocks
// (in block order) runs on one XCD, its blocks dispatched 8 workgroups apart,
// while the 8 XCDs work on neighbouring groups at the same time.  Halos inside
// a group meet in the XCD's L2, halos between groups in the shared
// last-level cache.  Needs nwg divisible by 8m (a bijection of [0, nwg)).
__host__ __device__ __forceinline__ int group_remap(int w, int m) {
  const int x = w & 7, r = (w >> 3) % m, i = w / (8 * m);
  return i * 8 * m + x * m + r;
}

// index of component 0 of slot s of block B, field with C components
__host__ __device__ __forceinline__ long fidx(const Geom& g, int B, int s, int C) {
  return ((long)B * (g.bs / TILE) + (s / TILE)) * C * TILE + (s % TILE);
}
// same for a field that lives on the odd slots only (io = s - half)
__host__ __device__ __forceinline__ long oidx(const Geom& g, int B, int io, int C) {
  return ((long)B * (g.half / TILE) + (io / TILE)) * C * TILE + (io % TILE);
}

__host__ __device__ __forceinline__ long lex_index(const Geom& g, const int x[4]) {
  return (((long)x[0] * g.L[1] + x[1]) * g.L[2] + x[2]) * g.L[3] + x[3];
}

// ---- host-side error types ------------------------------------------------
struct HipError : std::runtime_error {
  hipError_t code;
  HipError(hipError_t e, const char* expr, const char* file, int line)
      : std::runtime_error(std::string(hipGetErrorString(e)) + " in " + expr + " (" + file + ":" +
                           std::to_string(line) + ")"),
        code(e) {}
};

// status codes of the C ABI
enum Status { OK = 0, NOT_CONVERGED = 1, INVALID_ARG = -1, BAD_STATE = -2, HIP_FAIL = -3, OUT_OF_MEMORY = -4, NUMERICAL = -5 };

struct Error : std::runtime_error {
  int status;
  Error(int st, const std::string& msg) : std::runtime_error(msg), status(st) {}
};

}  // namespace ddamg

#define HIP_CHECK(expr)                                                          \
  do {                                                                           \
    hipError_t _e = (expr);                                                      \
    if (_e != hipSuccess) throw ::ddamg::HipError(_e, #expr, __FILE__, __LINE__); \
  } while (0)
