// Cyclic two-sided Jacobi for a small real symmetric matrix held in LDS,
// executed by one workgroup of NT threads.  Pairs follow the round-robin
// (circle) ordering so the rotations of one round are disjoint; a rotation
// is applied only when |M_pq| > tiny, and the sweep loop stops after a
// sweep with no rotation.  On exit diag(M) holds the eigenvalues and V the
// eigenvectors (M_out = V^T M_in V).
#pragma once
#include "common.hpp"

namespace ppcg {

PPCG_DEV int rr_player(int pos, int round, int rr) {
  return pos == 0 ? 0 : ((pos - 1 + round) % (rr - 1)) + 1;
}

template <int NT>
PPCG_DEV void lds_jacobi(double* M, double* V, int r, int LD, double tiny, int maxsweeps, double* cs, int* pq,
                         int* cnt) {
  const int tid = threadIdx.x;
  const int rr = r + (r & 1);
  const int np = rr / 2;
  for (int e = tid; e < r * r; e += NT) {
    int i = e % r, j = e / r;
    V[i + j * LD] = (i == j) ? 1.0 : 0.0;
  }
  if (r <= 1) {
    __syncthreads();
    return;
  }
  for (int sweep = 0; sweep < maxsweeps; ++sweep) {
    if (tid == 0) *cnt = 0;
    __syncthreads();
    for (int round = 0; round < rr - 1; ++round) {
      if (tid < np) {
        int a = rr_player(tid, round, rr), b = rr_player(rr - 1 - tid, round, rr);
        int p = a < b ? a : b, q = a < b ? b : a;
        double c = 1.0, s = 0.0;
        int act = 0;
        if (q < r) {
          double apq = M[p + q * LD];
          if (fabs(apq) > tiny) {
            double th = (M[q + q * LD] - M[p + p * LD]) / (2.0 * apq);
            double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
            act = 1;
          }
        }
        pq[2 * tid] = act ? p : -1;
        pq[2 * tid + 1] = q;
        cs[2 * tid] = c;
        cs[2 * tid + 1] = s;
        if (act) atomicAdd(cnt, 1);
      }
      __syncthreads();
      // rows p, q  <-  J^T M
      for (int w = tid; w < np * r; w += NT) {
        int t = w / r, j = w % r;
        int p = pq[2 * t];
        if (p < 0) continue;
        int q = pq[2 * t + 1];
        double c = cs[2 * t], s = cs[2 * t + 1];
        double mp = M[p + j * LD], mq = M[q + j * LD];
        M[p + j * LD] = c * mp - s * mq;
        M[q + j * LD] = s * mp + c * mq;
      }
      __syncthreads();
      // columns p, q  <-  M J ;  V <- V J
      for (int w = tid; w < np * r; w += NT) {
        int t = w / r, i = w % r;
        int p = pq[2 * t];
        if (p < 0) continue;
        int q = pq[2 * t + 1];
        double c = cs[2 * t], s = cs[2 * t + 1];
        double mp = M[i + p * LD], mq = M[i + q * LD];
        M[i + p * LD] = c * mp - s * mq;
        M[i + q * LD] = s * mp + c * mq;
        double vp = V[i + p * LD], vq = V[i + q * LD];
        V[i + p * LD] = c * vp - s * vq;
        V[i + q * LD] = s * vp + c * vq;
      }
      __syncthreads();
    }
    if (*cnt == 0) break;
    __syncthreads();
  }
  __syncthreads();
}

}  // namespace ppcg
