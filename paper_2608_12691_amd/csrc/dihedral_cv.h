// Dihedral collective variables and the d-AFED coupling (eq. 15) as the work
// of one thread block, shared by the CV launch (k_dihedrals) and by the
// lambda-dynamics step that evaluates the CVs in the same launch as the
// auxiliary-variable update.  FP64 throughout.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include "anb_internal.h"

namespace anb {
namespace dcv {

struct V3 {
  double x, y, z;
};
__device__ inline V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ inline V3 add(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ inline V3 scl(V3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
__device__ inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }

// Dihedral of r1..r4 (F = r1 - r2, G = r2 - r3, H = r4 - r3, plane normals
// A = F x G, B = H x G), xi = atan2((B x A).G/|G|, A.B) in (-pi, pi], and its
// Cartesian gradient written from the geometry of a torsion: an end atom
// moves xi only through the rotation of its plane about the axis, at rate
// |G|/|A|^2 (atom 1, along -A) and |G|/|B|^2 (atom 4, along +B); the two axis
// atoms then take the shares fixed by translation and rotation invariance,
// i.e. sum_i dxi/dr_i = 0 and sum_i r_i x dxi/dr_i = 0, which with the axial
// offsets f = F.G/|G|^2 and h = H.G/|G|^2 of the end atoms gives
//   dxi/dr2 = -(1 + f) dxi/dr1 - h dxi/dr4,  dxi/dr3 = f dxi/dr1 + (h - 1) dxi/dr4.
__device__ inline double dihedral_grad(V3 F, V3 G, V3 H, V3 g[4]) {
  const V3 A = cross(F, G), B = cross(H, G);
  const double gg = dot(G, G), gn = sqrt(gg);
  const double y = dot(cross(B, A), G) / gn, x = dot(A, B);
  const double xi = atan2(y, x);
  const double aa = dot(A, A), bb = dot(B, B);
  const V3 g1 = scl(A, -gn / aa);
  const V3 g4 = scl(B, gn / bb);
  const double f = dot(F, G) / gg, h = dot(H, G) / gg;
  g[0] = g1;
  g[3] = g4;
  g[1] = sub(scl(g1, -(1.0 + f)), scl(g4, h));
  g[2] = add(scl(g1, f), scl(g4, h - 1.0));
  return xi;
}

__device__ inline double mi1(double v, double L) { return v - L * rint(v / L); }

// Outputs of the CV pass; every pointer may be null.
struct CvOut {
  double* xi;              // [n_cv]
  double* dxi;             // [n_cv][4][3]
  const double* mass_inv;  // [n_atoms], with msum: sum_i m_i^-1 |dxi/dr_i|^2 (eq. 16)
  double* msum;            // [n_cv]
  double* u_dafed;         // [1], sum_c kappa_c wrap(xi_c - s_c)^2 / 2
  double* forces;          // [n_atoms][3], the coupling force added
};

// All CVs of d_idx [n_cv][4] by one block of kB threads, kB/4 CVs at a time.
// Per chunk: one thread per CV computes xi, its gradient and (with s and
// kappa) the coupling kappa wrap(xi - s); then one thread per distinct atom
// of the chunk adds that atom's coupling forces in the order of the atom's
// entries in d_idx (CV, then position in the quadruple), so each force
// component receives the same sequence of operations as a serial scatter
// over the CVs would give it, whatever the block size.  An index outside
// [0, n_atoms) raises flag 64 and leaves that CV's outputs unwritten.
// per_cv(c, valid, xi) is called by the CV's thread after its outputs are
// written (the lambda-dynamics step advances s_c there).
template <int kB, class PerCv>
__device__ inline void cv_block(const double* __restrict__ pos, int n_cv, const int* __restrict__ idx,
                                const double* s, const double* kappa, const CvOut& o, const ReplicaInfo* reps,
                                const int* atom_rep, int n_atoms, unsigned int* flags, PerCv per_cv) {
  static_assert(kB % 64 == 0 && kB >= 64, "whole waves");
  constexpr int kC = kB / 4;  // CVs per chunk: one entry of the chunk per thread
  __shared__ int e_atom[kB];
  __shared__ double e_g[kB][3];
  __shared__ double c_dw[kC];
  __shared__ double c_du[kC];
  const bool couple = s && kappa;
  const int t = threadIdx.x;
  double u_acc = 0.0;  // thread 0: the coupling energy, CVs in order
  for (int c0 = 0; c0 < n_cv; c0 += kC) {
    const int nc = min(kC, n_cv - c0);
    if (t < kC) {
      const int c = c0 + t;
      double du = 0.0, d_wrap = 0.0;
      V3 g[4] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
      int a[4] = {-1, -1, -1, -1};
      bool ok = t < nc;
      if (ok) {
        for (int j = 0; j < 4; ++j) {
          a[j] = idx[4 * c + j];
          ok = ok && a[j] >= 0 && a[j] < n_atoms;
        }
        if (!ok) atomicOr(flags, 64u);  // invalid atom index: CV skipped
      }
      double xi = 0.0;
      if (ok) {
        const ReplicaInfo& rp = reps[atom_rep[a[1]]];
        V3 r[4];
        for (int j = 0; j < 4; ++j) r[j] = {pos[3 * a[j]], pos[3 * a[j] + 1], pos[3 * a[j] + 2]};
        V3 F = sub(r[0], r[1]), G = sub(r[1], r[2]), H = sub(r[3], r[2]);
        F = {mi1(F.x, rp.box[0]), mi1(F.y, rp.box[1]), mi1(F.z, rp.box[2])};
        G = {mi1(G.x, rp.box[0]), mi1(G.y, rp.box[1]), mi1(G.z, rp.box[2])};
        H = {mi1(H.x, rp.box[0]), mi1(H.y, rp.box[1]), mi1(H.z, rp.box[2])};
        xi = dihedral_grad(F, G, H, g);
        if (o.xi) o.xi[c] = xi;
        if (o.dxi)
          for (int j = 0; j < 4; ++j) {
            o.dxi[12 * c + 3 * j] = g[j].x;
            o.dxi[12 * c + 3 * j + 1] = g[j].y;
            o.dxi[12 * c + 3 * j + 2] = g[j].z;
          }
        if (o.mass_inv && o.msum) {
          double m = 0.0;
          for (int j = 0; j < 4; ++j) m += o.mass_inv[a[j]] * dot(g[j], g[j]);
          o.msum[c] = m;
        }
        if (couple) {
          // periodic angular displacement wrapped into (-pi, pi]
          double dd = xi - s[c];
          dd = dd - 2.0 * M_PI * floor((dd + M_PI) / (2.0 * M_PI));
          if (dd == -M_PI) dd = M_PI;
          d_wrap = kappa[c] * dd;
          du = 0.5 * kappa[c] * dd * dd;
        }
      }
      if (t < nc) per_cv(c, ok, xi);
      for (int j = 0; j < 4; ++j) {
        e_atom[4 * t + j] = ok ? a[j] : -1;
        e_g[4 * t + j][0] = g[j].x;
        e_g[4 * t + j][1] = g[j].y;
        e_g[4 * t + j][2] = g[j].z;
      }
      c_dw[t] = d_wrap;
      c_du[t] = du;
    }
    __syncthreads();
    if (t == 0 && couple)
      for (int k = 0; k < nc; ++k) u_acc += c_du[k];
    if (o.forces && couple && t < 4 * nc) {
      const int a = e_atom[t];
      bool first = a >= 0;
      for (int e = 0; e < t && first; ++e) first = e_atom[e] != a;
      if (first) {
        double fx = o.forces[3 * a], fy = o.forces[3 * a + 1], fz = o.forces[3 * a + 2];
        for (int e = t; e < 4 * nc; ++e) {
          if (e_atom[e] != a) continue;
          const double dw = c_dw[e >> 2];
          fx -= dw * e_g[e][0];
          fy -= dw * e_g[e][1];
          fz -= dw * e_g[e][2];
        }
        o.forces[3 * a] = fx;
        o.forces[3 * a + 1] = fy;
        o.forces[3 * a + 2] = fz;
      }
    }
    // this chunk's force stores are seen by the next chunk's loads
    __syncthreads();
  }
  if (t == 0 && couple && o.u_dafed) o.u_dafed[0] = u_acc;
}

}  // namespace dcv
}  // namespace anb
