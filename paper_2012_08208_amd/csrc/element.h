// Element-level arithmetic of the P1 Galerkin operator (Sec. 3.1, eq. fe_form)
// for the isotropic law sigma = lambda tr(eps) I + 2 mu eps (Sec. 4.2,
// eq. stress).  P1 strains are constant per cell, so the element force is
// f_a = |T| E sigma(u) grad N_a exactly.
//
// On the unit grid every shape gradient has entries in {0, +-1}:
// * 3D Kuhn tetrahedron of permutation pi (corners c = cx + 2 cy + 4 cz of
//   the unit cube): the vertices are 0, e_pi0, e_pi0 + e_pi1, 7 and
//   grad u has columns u(v1)-u(v0), u(v2)-u(v1), u(v3)-u(v2) along
//   pi0, pi1, pi2; the vertex gradients are -e_pi0, e_pi0 - e_pi1,
//   e_pi1 - e_pi2, e_pi2.
// * 2D triangles (corners c = cx + 2 cy of the unit square) take their
//   gradients from the template arguments.
#pragma once

#include <hip/hip_runtime.h>

namespace topo {

template <typename T, int P0, int P1, int P2>
__device__ __forceinline__ void tet_force(const T (&u)[8][3], T lam, T mu, T (&f)[8][3]) {
  constexpr int c1 = 1 << P0;
  constexpr int c2 = c1 | (1 << P1);
  T G[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    G[a][P0] = u[c1][a] - u[0][a];
    G[a][P1] = u[c2][a] - u[c1][a];
    G[a][P2] = u[7][a] - u[c2][a];
  }
  const T tr = G[0][0] + G[1][1] + G[2][2];
  const T lt = lam * tr;
  const T m2 = mu + mu;
  T S[3][3];
  S[0][0] = lt + m2 * G[0][0];
  S[1][1] = lt + m2 * G[1][1];
  S[2][2] = lt + m2 * G[2][2];
  S[0][1] = S[1][0] = mu * (G[0][1] + G[1][0]);
  S[0][2] = S[2][0] = mu * (G[0][2] + G[2][0]);
  S[1][2] = S[2][1] = mu * (G[1][2] + G[2][1]);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    f[0][a] -= S[a][P0];
    f[c1][a] += S[a][P0] - S[a][P1];
    f[c2][a] += S[a][P1] - S[a][P2];
    f[7][a] += S[a][P2];
  }
}

// Strain energy u^T K0 u of one Kuhn tetrahedron at unit modulus divided by
// |T|: lambda tr(eps)^2 + 2 mu eps:eps (= 2 psi).
template <typename T, int P0, int P1, int P2>
__device__ __forceinline__ T tet_energy(const T (&u)[8][3], T lam, T mu) {
  constexpr int c1 = 1 << P0;
  constexpr int c2 = c1 | (1 << P1);
  T G[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    G[a][P0] = u[c1][a] - u[0][a];
    G[a][P1] = u[c2][a] - u[c1][a];
    G[a][P2] = u[7][a] - u[c2][a];
  }
  const T tr = G[0][0] + G[1][1] + G[2][2];
  const T e01 = 0.5 * (G[0][1] + G[1][0]);
  const T e02 = 0.5 * (G[0][2] + G[2][0]);
  const T e12 = 0.5 * (G[1][2] + G[2][1]);
  const T ee = G[0][0] * G[0][0] + G[1][1] * G[1][1] + G[2][2] * G[2][2] +
               2.0 * (e01 * e01 + e02 * e02 + e12 * e12);
  return lam * tr * tr + 2.0 * mu * ee;
}

template <typename T, int C0, int X0, int Y0, int C1, int X1, int Y1, int C2, int X2, int Y2>
__device__ __forceinline__ void tri_force(const T (&u)[4][2], T lam, T mu, T (&f)[4][2]) {
  T G[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    G[a][0] = T(X0) * u[C0][a] + T(X1) * u[C1][a] + T(X2) * u[C2][a];
    G[a][1] = T(Y0) * u[C0][a] + T(Y1) * u[C1][a] + T(Y2) * u[C2][a];
  }
  const T lt = lam * (G[0][0] + G[1][1]);
  const T S00 = lt + 2 * mu * G[0][0];
  const T S11 = lt + 2 * mu * G[1][1];
  const T S01 = mu * (G[0][1] + G[1][0]);
  f[C0][0] += T(X0) * S00 + T(Y0) * S01;
  f[C0][1] += T(X0) * S01 + T(Y0) * S11;
  f[C1][0] += T(X1) * S00 + T(Y1) * S01;
  f[C1][1] += T(X1) * S01 + T(Y1) * S11;
  f[C2][0] += T(X2) * S00 + T(Y2) * S01;
  f[C2][1] += T(X2) * S01 + T(Y2) * S11;
}

template <typename T, int C0, int X0, int Y0, int C1, int X1, int Y1, int C2, int X2, int Y2>
__device__ __forceinline__ T tri_energy(const T (&u)[4][2], T lam, T mu) {
  T G[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    G[a][0] = T(X0) * u[C0][a] + T(X1) * u[C1][a] + T(X2) * u[C2][a];
    G[a][1] = T(Y0) * u[C0][a] + T(Y1) * u[C1][a] + T(Y2) * u[C2][a];
  }
  const T tr = G[0][0] + G[1][1];
  const T e01 = 0.5 * (G[0][1] + G[1][0]);
  return lam * tr * tr + 2.0 * mu * (G[0][0] * G[0][0] + G[1][1] * G[1][1] + 2.0 * e01 * e01);
}

// The two triangles of a unit square.  Diagonal A joins corners 0 and 3:
// t0 = {0,1,3}, t1 = {0,3,2}; diagonal B joins corners 1 and 2:
// t0 = {0,1,2}, t1 = {1,3,2}.
template <typename T>
__device__ __forceinline__ void square_force(bool diag_a, const T (&u)[4][2], T l0, T m0, T l1, T m1,
                                             T (&f)[4][2]) {
  if (diag_a) {
    tri_force<T, 0, -1, 0, 1, 1, -1, 3, 0, 1>(u, l0, m0, f);
    tri_force<T, 0, 0, -1, 2, -1, 1, 3, 1, 0>(u, l1, m1, f);
  } else {
    tri_force<T, 0, -1, -1, 1, 1, 0, 2, 0, 1>(u, l0, m0, f);
    tri_force<T, 3, 1, 1, 1, 0, -1, 2, -1, 0>(u, l1, m1, f);
  }
}

template <typename T>
__device__ __forceinline__ void square_energy(bool diag_a, const T (&u)[4][2], T lam, T mu, T& w0,
                                              T& w1) {
  if (diag_a) {
    w0 = tri_energy<T, 0, -1, 0, 1, 1, -1, 3, 0, 1>(u, lam, mu);
    w1 = tri_energy<T, 0, 0, -1, 2, -1, 1, 3, 1, 0>(u, lam, mu);
  } else {
    w0 = tri_energy<T, 0, -1, -1, 1, 1, 0, 2, 0, 1>(u, lam, mu);
    w1 = tri_energy<T, 3, 1, 1, 1, 0, -1, 2, -1, 0>(u, lam, mu);
  }
}

// Stress of one Kuhn tetrahedron (scaled by |T| E through lam, mu) from
// the three edge differences along its path: column pi_k of grad u is
// the k-th path edge.
template <typename T, int P0, int P1, int P2>
__device__ __forceinline__ void tet_stress(const T (&a)[3], const T (&b)[3], const T (&c)[3], T lam,
                                           T mu, T (&S)[3][3]) {
  T G[3][3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    G[k][P0] = a[k];
    G[k][P1] = b[k];
    G[k][P2] = c[k];
  }
  const T lt = lam * (G[0][0] + G[1][1] + G[2][2]);
  const T m2 = mu + mu;
  S[0][0] = lt + m2 * G[0][0];
  S[1][1] = lt + m2 * G[1][1];
  S[2][2] = lt + m2 * G[2][2];
  S[0][1] = S[1][0] = mu * (G[0][1] + G[1][0]);
  S[0][2] = S[2][0] = mu * (G[0][2] + G[2][0]);
  S[1][2] = S[2][1] = mu * (G[1][2] + G[2][1]);
}

// Forces of the six Kuhn tetrahedra of a unit cube on its 8 corners.
// Tetrahedron t (permutation pi) has path 0 -> e_pi0 -> e_pi0+e_pi1 -> 7 and
// vertex gradients -e_pi0, e_pi0 - e_pi1, e_pi1 - e_pi2, e_pi2, so corner
// forces are signed sums of stress columns; each corner's sum is formed
// once (assignments, no zero-initialised accumulators).
template <typename T>
__device__ __forceinline__ void cube_force(const T (&u)[8][3], const T (&lam)[6], const T (&mu)[6],
                                           T (&f)[8][3]) {
  T e01[3], e02[3], e04[3], e13[3], e15[3], e23[3], e26[3], e45[3], e46[3], e37[3], e57[3], e67[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    e01[k] = u[1][k] - u[0][k];
    e02[k] = u[2][k] - u[0][k];
    e04[k] = u[4][k] - u[0][k];
    e13[k] = u[3][k] - u[1][k];
    e15[k] = u[5][k] - u[1][k];
    e23[k] = u[3][k] - u[2][k];
    e26[k] = u[6][k] - u[2][k];
    e45[k] = u[5][k] - u[4][k];
    e46[k] = u[6][k] - u[4][k];
    e37[k] = u[7][k] - u[3][k];
    e57[k] = u[7][k] - u[5][k];
    e67[k] = u[7][k] - u[6][k];
  }
  T S0[3][3], S1[3][3], S2[3][3], S3[3][3], S4[3][3], S5[3][3];
  tet_stress<T, 0, 1, 2>(e01, e13, e37, lam[0], mu[0], S0);  // 0-1-3-7
  tet_stress<T, 0, 2, 1>(e01, e15, e57, lam[1], mu[1], S1);  // 0-1-5-7
  tet_stress<T, 1, 0, 2>(e02, e23, e37, lam[2], mu[2], S2);  // 0-2-3-7
  tet_stress<T, 1, 2, 0>(e02, e26, e67, lam[3], mu[3], S3);  // 0-2-6-7
  tet_stress<T, 2, 0, 1>(e04, e45, e57, lam[4], mu[4], S4);  // 0-4-5-7
  tet_stress<T, 2, 1, 0>(e04, e46, e67, lam[5], mu[5], S5);  // 0-4-6-7
  // Corner sums share their partial sums: tetrahedra 0,1 / 2,3 / 4,5 leave
  // corner 0 along x / y / z (column pi0 of their stress), and the pairs
  // meeting at corners 3, 5, 6 (e_pi0 + e_pi1) enter corner 7 along the
  // same axis (column pi2).
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const T ax = S0[k][0] + S1[k][0];   // column pi0 of the tets leaving along x
    const T ay = S2[k][1] + S3[k][1];   // ... along y
    const T az = S4[k][2] + S5[k][2];   // ... along z
    const T c3 = S0[k][2] + S2[k][2];   // column pi2 of the tets through corner 3
    const T c5 = S1[k][1] + S4[k][1];   // ... through corner 5
    const T c6 = S3[k][0] + S5[k][0];   // ... through corner 6
    f[0][k] = -((ax + ay) + az);
    f[7][k] = (c3 + c5) + c6;
    // corners e_pi0: S[:, pi0] - S[:, pi1]
    f[1][k] = ax - (S0[k][1] + S1[k][2]);
    f[2][k] = ay - (S2[k][0] + S3[k][2]);
    f[4][k] = az - (S4[k][0] + S5[k][1]);
    // corners e_pi0 + e_pi1: S[:, pi1] - S[:, pi2]
    f[3][k] = (S0[k][1] + S2[k][0]) - c3;
    f[5][k] = (S1[k][2] + S4[k][0]) - c5;
    f[6][k] = (S3[k][2] + S5[k][1]) - c6;
  }
}

template <typename T>
__device__ __forceinline__ void cube_energy(const T (&u)[8][3], T lam, T mu, T (&w)[6]) {
  w[0] = tet_energy<T, 0, 1, 2>(u, lam, mu);
  w[1] = tet_energy<T, 0, 2, 1>(u, lam, mu);
  w[2] = tet_energy<T, 1, 0, 2>(u, lam, mu);
  w[3] = tet_energy<T, 1, 2, 0>(u, lam, mu);
  w[4] = tet_energy<T, 2, 0, 1>(u, lam, mu);
  w[5] = tet_energy<T, 2, 1, 0>(u, lam, mu);
}

}  // namespace topo
