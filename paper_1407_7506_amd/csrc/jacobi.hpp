// Cyclic two-sided Jacobi for a small real symmetric matrix held in LDS,
// executed by one workgroup of NT threads.  Pairs follow the round-robin
// (circle) ordering, so the rotations of one round are disjoint and the
// two-sided update J^T M J splits into independent 2x2 blocks
// (rows of pair a, columns of pair b): one pass per round.  A rotation is
// applied only when |M_pq| > tiny; the sweep loop stops after a sweep with
// no rotation.  On exit diag(M) holds the eigenvalues and V the
// eigenvectors (M_out = V^T M_in V).
#pragma once
#include "common.hpp"

namespace ppcg {

PPCG_DEV int rr_player(int pos, int round, int rr) {
  return pos == 0 ? 0 : ((pos - 1 + round) % (rr - 1)) + 1;
}

// cs: 2*(r+1)/2 doubles, pq: 2*(r+1)/2 ints (LDS)
template <int NT>
PPCG_DEV int lds_jacobi(double* M, double* V, int r, int LD, double tiny, int maxsweeps, double* cs, int* pq,
                        int* cnt) {
  const int tid = threadIdx.x;
  const int rr = r + (r & 1);
  const int np = rr / 2;
  for (int e = tid; e < r * r; e += NT) {
    int i = e % r, j = e / r;
    V[i + j * LD] = (i == j) ? 1.0 : 0.0;
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
        if (q < r) {
          double apq = M[p + q * LD];
          if (fabs(apq) > tiny) {
            double th = (M[q + q * LD] - M[p + p * LD]) / (2.0 * apq);
            double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
            atomicAdd(cnt, 1);
          }
        }
        pq[2 * tid] = p;
        pq[2 * tid + 1] = q;
        cs[2 * tid] = c;
        cs[2 * tid + 1] = s;
      }
      __syncthreads();
      // 2x2 blocks: rows {p_a, q_a} x columns {p_b, q_b}
      for (int w = tid; w < np * np; w += NT) {
        int ta = w % np, tb = w / np;
        double ca = cs[2 * ta], sa = cs[2 * ta + 1], cb = cs[2 * tb], sb = cs[2 * tb + 1];
        if (sa == 0.0 && sb == 0.0) continue;
        int p = pq[2 * ta], q = pq[2 * ta + 1], p2 = pq[2 * tb], q2 = pq[2 * tb + 1];
        bool vq = q < r, vq2 = q2 < r;
        double b00 = M[p + p2 * LD];
        double b01 = vq2 ? M[p + q2 * LD] : 0.0;
        double b10 = vq ? M[q + p2 * LD] : 0.0;
        double b11 = (vq && vq2) ? M[q + q2 * LD] : 0.0;
        double r00 = ca * b00 - sa * b10, r10 = sa * b00 + ca * b10;
        double r01 = ca * b01 - sa * b11, r11 = sa * b01 + ca * b11;
        M[p + p2 * LD] = cb * r00 - sb * r01;
        if (vq2) M[p + q2 * LD] = sb * r00 + cb * r01;
        if (vq) M[q + p2 * LD] = cb * r10 - sb * r11;
        if (vq && vq2) M[q + q2 * LD] = sb * r10 + cb * r11;
      }
      // V <- V J (columns of each rotated pair)
      for (int w = tid; w < r * np; w += NT) {
        int i = w % r, tb = w / r;
        double sb = cs[2 * tb + 1];
        if (sb == 0.0) continue;
        double cb = cs[2 * tb];
        int p2 = pq[2 * tb], q2 = pq[2 * tb + 1];
        double vp = V[i + p2 * LD], vq = V[i + q2 * LD];
        V[i + p2 * LD] = cb * vp - sb * vq;
        V[i + q2 * LD] = sb * vp + cb * vq;
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
