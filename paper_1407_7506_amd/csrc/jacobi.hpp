// Cyclic two-sided Jacobi for a small Hermitian matrix (in LDS, or in device
// memory for the largest block pencils), executed by one workgroup of NT
// threads.  Pairs follow the round-robin (circle) ordering, so the rotations
// of one round are disjoint and the two-sided update J^H M J splits into
// independent 2x2 blocks (rows of pair a, columns of pair b): one pass per
// round.  With M_pq = |M_pq| u the rotation is
// J = [[c, s], [-s conj(u), c conj(u)]] (a phase that makes M_pq real and
// positive, then a real rotation); for real data u is the sign of M_pq.  A
// rotation is applied only when |M_pq| > tiny; the sweep loop stops after a
// sweep with no rotation.  On exit the real parts of diag(M) hold the
// eigenvalues and V the eigenvectors (M_out = V^H M_in V).
#pragma once
#include "common.hpp"

namespace ppcg {

PPCG_DEV int rr_player(int pos, int round, int rr) {
  return pos == 0 ? 0 : ((pos - 1 + round) % (rr - 1)) + 1;
}

// u = M_pq / |M_pq|: a unit complex number, or the sign (+1 / -1) for real data
template <class S> PPCG_DEV S unit_phase(S a, double mag) {
  if constexpr (sc_traits<S>::cplx) return S{a.x / mag, a.y / mag};
  else return a >= 0 ? (S)1.0 : (S)-1.0;
}
template <class S> PPCG_DEV double mag_(S a) {
  if constexpr (sc_traits<S>::cplx) return sqrt(abs2_(a));
  else return fabs(a);
}
// z * u for u a unit phase (real data: u = +1 or -1)
template <class S> PPCG_DEV S mulu(S z, S u) {
  return z * u;
}

// cs: 2*(r+1)/2 doubles, uu: (r+1)/2 scalars, pq: 2*(r+1)/2 ints (all LDS)
template <int NT, class S>
PPCG_DEV int lds_jacobi(S* M, S* V, int r, int LD, double tiny, int maxsweeps, double* cs, S* uu, int* pq, int* cnt) {
  const int tid = threadIdx.x;
  const int rr = r + (r & 1);
  const int np = rr / 2;
  for (int e = tid; e < r * r; e += NT) {
    int i = e % r, j = e / r;
    V[i + j * LD] = from_real<S>(i == j ? 1.0 : 0.0);
  }
  int sweeps = 0;
  if (r <= 1) {
    __syncthreads();
    return 0;
  }
  for (int sweep = 0; sweep < maxsweeps; ++sweep) {
    if (tid == 0) *cnt = 0;
    __syncthreads();
    for (int round = 0; round < rr - 1; ++round) {
      if (tid < np) {
        int a = rr_player(tid, round, rr), b = rr_player(rr - 1 - tid, round, rr);
        int p = a < b ? a : b, q = a < b ? b : a;
        double c = 1.0, s = 0.0;
        S u = from_real<S>(1.0);
        if (q < r) {
          S apq = M[p + q * LD];
          double mag = mag_(apq);
          if (mag > tiny) {
            double th = (real_(M[q + q * LD]) - real_(M[p + p * LD])) / (2.0 * mag);
            double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
            u = unit_phase(apq, mag);
            atomicAdd(cnt, 1);
          }
        }
        pq[2 * tid] = p;
        pq[2 * tid + 1] = q;
        cs[2 * tid] = c;
        cs[2 * tid + 1] = s;
        uu[tid] = u;
      }
      __syncthreads();
      // 2x2 blocks: rows {p_a, q_a} x columns {p_b, q_b}:  J_a^H B J_b
      for (int w = tid; w < np * np; w += NT) {
        int ta = w % np, tb = w / np;
        double ca = cs[2 * ta], sa = cs[2 * ta + 1], cb = cs[2 * tb], sb = cs[2 * tb + 1];
        if (sa == 0.0 && sb == 0.0) continue;
        S ua = uu[ta], ub = conj_(uu[tb]);
        int p = pq[2 * ta], q = pq[2 * ta + 1], p2 = pq[2 * tb], q2 = pq[2 * tb + 1];
        bool vq = q < r, vq2 = q2 < r;
        S zero = from_real<S>(0.0);
        S b00 = M[p + p2 * LD];
        S b01 = vq2 ? M[p + q2 * LD] : zero;
        S b10 = vq ? M[q + p2 * LD] : zero;
        S b11 = (vq && vq2) ? M[q + q2 * LD] : zero;
        // rows: (J^H)_p = [c, -s u], (J^H)_q = [s, c u]
        S r00 = ca * b00 - sa * mulu(b10, ua), r10 = sa * b00 + ca * mulu(b10, ua);
        S r01 = ca * b01 - sa * mulu(b11, ua), r11 = sa * b01 + ca * mulu(b11, ua);
        // columns: J_p = [c, -s conj(u)]^T, J_q = [s, c conj(u)]^T
        M[p + p2 * LD] = cb * r00 - sb * mulu(r01, ub);
        if (vq2) M[p + q2 * LD] = sb * r00 + cb * mulu(r01, ub);
        if (vq) M[q + p2 * LD] = cb * r10 - sb * mulu(r11, ub);
        if (vq && vq2) M[q + q2 * LD] = sb * r10 + cb * mulu(r11, ub);
      }
      // V <- V J (columns of each rotated pair)
      for (int w = tid; w < r * np; w += NT) {
        int i = w % r, tb = w / r;
        double sb = cs[2 * tb + 1];
        if (sb == 0.0) continue;
        double cb = cs[2 * tb];
        S ub = conj_(uu[tb]);
        int p2 = pq[2 * tb], q2 = pq[2 * tb + 1];
        S vp = V[i + p2 * LD], vq = V[i + q2 * LD];
        V[i + p2 * LD] = cb * vp - sb * mulu(vq, ub);
        V[i + q2 * LD] = sb * vp + cb * mulu(vq, ub);
      }
      __syncthreads();
    }
    ++sweeps;
    if (*cnt == 0) break;
    __syncthreads();
  }
  __syncthreads();
  return sweeps;
}

}  // namespace ppcg
