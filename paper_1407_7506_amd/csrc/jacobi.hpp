// Cyclic two-sided Jacobi for a small Hermitian matrix (in LDS, or in device
// memory for the largest block pencils), executed by one workgroup of NT
// threads.  Pairs follow the round-robin (circle) ordering, so the rotations
// of one round are disjoint and the two-sided update J^H M J splits into
// independent 2x2 blocks (rows of pair a, columns of pair b): one pass per
// round.  With M_pq = |M_pq| u the rotation is
// J = [[c, s], [-s conj(u), c conj(u)]] (a phase that makes M_pq real and
// positive, then a real rotation); for real data u is the sign of M_pq.  A
// rotation is applied only when |M_pq| > tiny; the sweep loop stops once no
// off-diagonal entry exceeds tiny.  On exit the real parts of diag(M) hold the
// eigenvalues and V the eigenvectors (M_out = V^H M_in V).
#pragma once
#include "common.hpp"

namespace ppcg {

PPCG_DEV int rr_player(int pos, int round, int rr) {
  return pos == 0 ? 0 : ((pos - 1 + round) % (rr - 1)) + 1;
}

template <class S> PPCG_DEV double mag_(S a) {
  if constexpr (sc_traits<S>::cplx) return sqrt(abs2_(a));
  else return fabs(a);
}
// z * u for u a unit phase (real data: u = +1 or -1)
template <class S> PPCG_DEV S mulu(S z, S u) {
  return z * u;
}

// Circle ordering without integer division: index at a position in a round
PPCG_DEV int rr_at(int pos, int round, int rr) {
  if (pos == 0) return 0;
  int x = pos - 1 + round;
  if (x >= rr - 1) x -= rr - 1;
  return x + 1;
}

// 1/sqrt(x) for finite x > 0: the hardware estimate refined by two Newton
// steps (each squares the relative error), i.e. to within a few ulp
PPCG_DEV double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const double e = fma(-x * y, y, 1.0);  // 1 - x y^2
    y = fma(0.5 * y, e, y);
  }
  return y;
}

// Rotation parameters of one pair: J as above, identity when off.  With
// d = a_qq - a_pp, r = sqrt(d^2 + 4 |a_pq|^2) and w = |d| + r, the tangent is
// t = sign(d) 2 |a_pq| / w, so c = w / sqrt(w^2 + 4 |a_pq|^2) and
// s = sign(d) 2 |a_pq| / sqrt(w^2 + 4 |a_pq|^2), where w^2 + 4 |a_pq|^2 = 2 r w:
// two refined reciprocal square roots instead of a chain of three divisions
// and two square roots (same rotation, to a few ulp).
template <class S> struct JRot {
  double c, s;
  S u;
  int on;
};
template <class S>
PPCG_DEV JRot<S> jacobi_rot(S apq, double app, double aqq, double tiny) {
  JRot<S> o;
  o.c = 1.0;
  o.s = 0.0;
  o.u = from_real<S>(1.0);
  o.on = 0;
  double mag, imag = 0.0;
  if constexpr (sc_traits<S>::cplx) {  // |a_pq| exactly as the sweep stop tests take it
    const double m2 = abs2_(apq);
    mag = sqrt(m2);
    imag = m2 > 0 ? rsqrt_nr(m2) : 0.0;
  } else {
    mag = fabs(apq);
  }
  if (mag > tiny) {
    const double d = aqq - app;
    const double q = fma(d, d, 4.0 * mag * mag);
    const double r = q * rsqrt_nr(q);
    const double w = fabs(d) + r;
    const double inv = rsqrt_nr(2.0 * r * w);
    o.c = w * inv;
    o.s = (d >= 0 ? 2.0 : -2.0) * mag * inv;
    if constexpr (sc_traits<S>::cplx) o.u = S{apq.x * imag, apq.y * imag};
    else o.u = apq >= 0 ? (S)1.0 : (S)-1.0;
    o.on = 1;
  }
  return o;
}
// J_a^H B J_b on the 2x2 block (b00 b01; b10 b11)
template <class S>
PPCG_DEV void jacobi_2x2(const JRot<S>& A, const JRot<S>& B, S& b00, S& b01, S& b10, S& b11) {
  const double ca = A.c, sa = A.s, cb = B.c, sb = B.s;
  const S ua = A.u, ub = conj_(B.u);
  // rows: (J^H)_p = [c, -s u], (J^H)_q = [s, c u]
  S r00 = ca * b00 - sa * mulu(b10, ua), r10 = sa * b00 + ca * mulu(b10, ua);
  S r01 = ca * b01 - sa * mulu(b11, ua), r11 = sa * b01 + ca * mulu(b11, ua);
  // columns: J_p = [c, -s conj(u)]^T, J_q = [s, c conj(u)]^T
  b00 = cb * r00 - sb * mulu(r01, ub);
  b01 = sb * r00 + cb * mulu(r01, ub);
  b10 = cb * r10 - sb * mulu(r11, ub);
  b11 = sb * r10 + cb * mulu(r11, ub);
}

// M: r x r (leading dimension LD), rotated in place; V: the eigenvectors;
// rot: (r+1)/2 rotation records; red: NT/64 doubles.  Per round, threads
// [0, np) form the rotations (barrier), then threads [0, np^2) apply the
// 2x2 blocks and the next ones a rotation pair of V over a stride of its
// rows (barrier).  After each sweep the largest off-diagonal magnitude
// decides exactly what a further sweep would do: with none above tiny it
// would rotate nothing, so the loop stops there.
template <int NT, class S>
PPCG_DEV int lds_jacobi(S* M, S* V, int r, int LD, double tiny, int maxsweeps, JRot<S>* rot, double* red) {
  const int tid = threadIdx.x;
  const int rr = r + (r & 1);
  const int np = rr / 2;
  for (int e = tid; e < r * r; e += NT) {
    int i = e % r, j = e / r;
    V[i + j * LD] = from_real<S>(i == j ? 1.0 : 0.0);
  }
  __syncthreads();
  if (r <= 1) return 0;
  const int nm = np * np;
  const bool split = nm + np <= NT;  // blocks and rows of V by different threads
  const int vbase = split ? nm : 0;
  const int vthr = (split ? NT - nm : NT) / np * np;
  const int rstep = vthr / np;
  const int mend = (split && tid >= nm) ? 0 : nm;
  int sweeps = 0;
  for (int sweep = 0; sweep < maxsweeps; ++sweep) {
    for (int round = 0; round < rr - 1; ++round) {
      for (int t = tid; t < np; t += NT) {
        int p = rr_at(t, round, rr), q = rr_at(rr - 1 - t, round, rr);
        if (p > q) { int x = p; p = q; q = x; }
        JRot<S> o{1.0, 0.0, from_real<S>(1.0), 0};
        if (q < r) o = jacobi_rot(M[p + q * LD], real_(M[p + p * LD]), real_(M[q + q * LD]), tiny);
        rot[t] = o;
      }
      __syncthreads();
      // 2x2 blocks: rows {p_a, q_a} x columns {p_b, q_b}:  J_a^H B J_b
      for (int w = tid; w < mend; w += NT) {
        const int ta = w % np, tb = w / np;
        const JRot<S> A = rot[ta], B = rot[tb];
        if (!A.on && !B.on) continue;
        int p = rr_at(ta, round, rr), q = rr_at(rr - 1 - ta, round, rr);
        if (p > q) { int x = p; p = q; q = x; }
        int p2 = rr_at(tb, round, rr), q2 = rr_at(rr - 1 - tb, round, rr);
        if (p2 > q2) { int x = p2; p2 = q2; q2 = x; }
        const bool vq = q < r, vq2 = q2 < r;
        const S zero = from_real<S>(0.0);
        S b00 = M[p + p2 * LD];
        S b01 = vq2 ? M[p + q2 * LD] : zero;
        S b10 = vq ? M[q + p2 * LD] : zero;
        S b11 = (vq && vq2) ? M[q + q2 * LD] : zero;
        jacobi_2x2(A, B, b00, b01, b10, b11);
        M[p + p2 * LD] = b00;
        if (vq2) M[p + q2 * LD] = b01;
        if (vq) M[q + p2 * LD] = b10;
        if (vq && vq2) M[q + q2 * LD] = b11;
      }
      // V <- V J (columns of each rotated pair)
      {
        const int vt = tid - vbase;
        if (vt >= 0 && vt < vthr) {
          const int tb = vt % np;
          const JRot<S> B = rot[tb];
          if (B.on) {
            int p2 = rr_at(tb, round, rr), q2 = rr_at(rr - 1 - tb, round, rr);
            if (p2 > q2) { int x = p2; p2 = q2; q2 = x; }
            const double cb = B.c, sb = B.s;
            const S ub = conj_(B.u);
            for (int i = vt / np; i < r; i += rstep) {
              S vp = V[i + p2 * LD], vq = V[i + q2 * LD];
              V[i + p2 * LD] = cb * vp - sb * mulu(vq, ub);
              V[i + q2 * LD] = sb * vp + cb * mulu(vq, ub);
            }
          }
        }
      }
      __syncthreads();
    }
    ++sweeps;
    if (sweep + 1 < maxsweeps) {
      double mx = 0;
      for (int e = tid; e < r * r; e += NT) {
        int i = e % r, j = e / r;
        if (i != j) mx = fmax(mx, mag_(M[i + j * LD]));
      }
      for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
      if ((tid & 63) == 0) red[tid >> 6] = mx;
      __syncthreads();
      mx = 0;
#pragma unroll
      for (int w = 0; w < NT / 64; ++w) mx = fmax(mx, red[w]);
      if (!(mx > tiny)) break;
    }
  }
  __syncthreads();
  return sweeps;
}

}  // namespace ppcg
