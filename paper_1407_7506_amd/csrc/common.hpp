// Shared device/host definitions for libppcg (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define PPCG_DEV __device__ __forceinline__

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

namespace ppcg {

// ---------------------------------------------------------------------------
// Scalars: real (double, float) or complex (cpx<double>, cpx<float>, stored
// interleaved re, im).  The same kernel templates serve both.
// ---------------------------------------------------------------------------
template <class R> struct cpx {
  R x, y;
};
typedef cpx<double> zdouble;
typedef cpx<float> zfloat;

template <class S> struct sc_traits { typedef S real_t; static constexpr bool cplx = false; };
template <class R> struct sc_traits<cpx<R>> { typedef R real_t; static constexpr bool cplx = true; };

template <class R> PPCG_DEV cpx<R> operator+(cpx<R> a, cpx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <class R> PPCG_DEV cpx<R> operator-(cpx<R> a, cpx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <class R> PPCG_DEV cpx<R> operator-(cpx<R> a) { return {-a.x, -a.y}; }
template <class R> PPCG_DEV cpx<R> operator*(cpx<R> a, cpx<R> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <class R> PPCG_DEV cpx<R> operator*(R s, cpx<R> a) { return {s * a.x, s * a.y}; }
template <class R> PPCG_DEV cpx<R> operator*(cpx<R> a, R s) { return {s * a.x, s * a.y}; }
template <class R> PPCG_DEV cpx<R> operator/(cpx<R> a, R s) { return {a.x / s, a.y / s}; }
template <class R> PPCG_DEV cpx<R>& operator+=(cpx<R>& a, cpx<R> b) { a.x += b.x; a.y += b.y; return a; }
template <class R> PPCG_DEV cpx<R>& operator-=(cpx<R>& a, cpx<R> b) { a.x -= b.x; a.y -= b.y; return a; }
template <class R> PPCG_DEV cpx<R>& operator*=(cpx<R>& a, R s) { a.x *= s; a.y *= s; return a; }
template <class R> PPCG_DEV cpx<R>& operator/=(cpx<R>& a, R s) { a.x /= s; a.y /= s; return a; }

PPCG_DEV double conj_(double a) { return a; }
PPCG_DEV float conj_(float a) { return a; }
template <class R> PPCG_DEV cpx<R> conj_(cpx<R> a) { return {a.x, -a.y}; }
PPCG_DEV double real_(double a) { return a; }
PPCG_DEV float real_(float a) { return a; }
template <class R> PPCG_DEV R real_(cpx<R> a) { return a.x; }
PPCG_DEV double abs2_(double a) { return a * a; }
PPCG_DEV float abs2_(float a) { return a * a; }
template <class R> PPCG_DEV R abs2_(cpx<R> a) { return a.x * a.x + a.y * a.y; }
template <class S> PPCG_DEV S from_real(typename sc_traits<S>::real_t r);
template <> PPCG_DEV double from_real<double>(double r) { return r; }
template <> PPCG_DEV float from_real<float>(float r) { return r; }
template <> PPCG_DEV zdouble from_real<zdouble>(double r) { return {r, 0.0}; }
template <> PPCG_DEV zfloat from_real<zfloat>(float r) { return {r, 0.0f}; }
// precision conversions (double <-> float, complex <-> complex)
template <class D, class S> PPCG_DEV D cvt(S a);
template <> PPCG_DEV double cvt<double, double>(double a) { return a; }
template <> PPCG_DEV double cvt<double, float>(float a) { return a; }
template <> PPCG_DEV float cvt<float, double>(double a) { return (float)a; }
template <> PPCG_DEV float cvt<float, float>(float a) { return a; }
template <> PPCG_DEV zdouble cvt<zdouble, zdouble>(zdouble a) { return a; }
template <> PPCG_DEV zdouble cvt<zdouble, zfloat>(zfloat a) { return {a.x, a.y}; }
template <> PPCG_DEV zfloat cvt<zfloat, zdouble>(zdouble a) { return {(float)a.x, (float)a.y}; }
template <> PPCG_DEV zfloat cvt<zfloat, zfloat>(zfloat a) { return a; }

// ---------------------------------------------------------------------------
// Workgroup index remap so that consecutive logical indices run on one XCD.
// The dispatcher places workgroup b on XCD (b mod 8); the logical index
// returned here groups the workgroups of each XCD into one contiguous range,
// so tiles that share operands (same row chunk / same row tile) share an L2.
// ---------------------------------------------------------------------------
PPCG_DEV unsigned xcd_remap(unsigned b, unsigned total) {
  const unsigned nx = 8;
  unsigned xcd = b % nx, idx = b / nx;
  unsigned per = total / nx, rem = total % nx;
  unsigned base = xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per;
  return base + idx;
}

// Grouped launches: one grid covers several jobs; job j owns workgroups
// [start[j], start[j+1]).  Returns the job of workgroup b (binary search for
// the last start <= b, so jobs with no workgroups are skipped).
PPCG_DEV int find_job(const unsigned* start, int nj, unsigned b) {
  int lo = 0, hi = nj - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// MFMA wrappers: 16x16x4 tiles.  Lane l supplies a = A[l%16][l/16] and
// b = B[l/16][l%16] (the reduction index is k = l/16).
//   f64: accumulator value v of lane l is D[4v + l/16][l%16]
//   f32: accumulator value v of lane l is D[4(l/16) + v][l%16]
PPCG_DEV d4v mfma(double a, double b, d4v c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
PPCG_DEV f4v mfma(float a, float b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <class T> struct AccT;
template <> struct AccT<double> { typedef d4v type; };
template <> struct AccT<float> { typedef f4v type; };

// Row (within a 16x16 tile) of accumulator value v in lane l.
template <class T> PPCG_DEV int acc_row(int l, int v);
template <> PPCG_DEV int acc_row<double>(int l, int v) { return 4 * v + (l >> 4); }
template <> PPCG_DEV int acc_row<float>(int l, int v) { return 4 * (l >> 4) + v; }

// Wave-level sum (64 lanes), deterministic butterfly order.
template <class T> PPCG_DEV T wave_sum(T v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

}  // namespace ppcg
