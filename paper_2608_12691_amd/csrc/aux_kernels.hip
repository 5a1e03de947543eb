// Backward pass, dihedral collective variables and the lambda/OPES update.
//
// - k_pgrad: a second pass over the list that sums, per atom type, the
//   derivatives of the pair energies with respect to sigma, sqrt(epsilon)
//   and the charge, weighted by the upstream gradient of each box.  Per-block
//   sums live in LDS (FP64 atomics), block partials are reduced in a fixed
//   order.  Pair inputs come from the FP64 positions (rounded once).
// - k_backward_finish: -g_k F and g_k dU/dlambda from the last forward.
// - k_dihedrals: dihedral angles, their Cartesian gradients (from the plane
//   rotation rates and the invariances, see dihedral_grad), the paper's
//   eq. 16 sum and the d-AFED coupling (eq. 15).
// - k_opes: mirror-periodic theta (eq. 3), dual OPES bias (eqs. 11-14),
//   kernel deposition, generalized force on theta.  FP64, one block.
#include <hip/hip_runtime.h>

#include "anb_internal.h"
#include "anb_kernels.h"
#include "erfc_coeffs.h"

namespace anb {

constexpr int kBlk = 256;

__device__ inline double local_x(const Dev& d, const double* __restrict__ x, int a, int s, int k, double L) {
  double m = x[3 * a + k] - d.x_build[3 * a + k];
  m -= L * rint(m / L);
  return m + (d.xw[3 * a + k] - d.sc_origin[3 * s + k]);
}

template <typename R>
__device__ inline R rsq_(R x);
template <>
__device__ inline float rsq_(float x) {
  return __builtin_amdgcn_rsqf(x);
}
template <>
__device__ inline double rsq_(double x) {
  return 1.0 / sqrt(x);
}
__device__ inline void erfc_exp_(float x, float& ec, float& ex) {
  const float t = __builtin_amdgcn_rcpf(fmaf(ANB_ERFC_P, x, 1.0f));
  float p = kErfcCoef[ANB_ERFC_DEG];
#pragma unroll
  for (int k = ANB_ERFC_DEG - 1; k >= 0; --k) p = fmaf(p, t, kErfcCoef[k]);
  ex = __builtin_amdgcn_exp2f((x * x) * -1.4426950408889634f);
  ec = t * p * ex;
}
__device__ inline void erfc_exp_(double x, double& ec, double& ex) {
  ex = exp(-x * x);
  ec = erfc(x);
}

// Derivatives of one pair energy with respect to the combined parameters
// sigma_ij, eps_ij and (q_i q_j) (raw charges).
template <typename R, int SCHED, bool SW>
__device__ inline void pair_param_derivs(R r2, bool alch, R sg, R e4, R inv_s6, R la0, R la1, const PotConsts& pc,
                                         R& dsig, R& deps, R& dqq) {
  const R rinv = rsq_<R>(r2), rinv2 = rinv * rinv, r = r2 * rinv;
  const R s2 = sg * sg * rinv2, s6 = s2 * s2 * s2;
  const R lj4 = R(4) * s6 * (s6 - R(1));            // dLJ/deps
  const R flj = e4 * s6 * (R(12) * s6 - R(6));      // sigma dLJ/dsigma = -r dLJ/dr
  R S = R(1);
  if (SW) {
    const R t = fmin(fmax((r - (R)pc.rs) * (R)pc.inv_w, R(0)), R(1));
    S = R(1) - t * t * t * (R(10) + t * (R(-15) + R(6) * t));
  }
  R ec, ex;
  erfc_exp_((R)pc.alpha * r, ec, ex);
  const R D = (R)kKe * (ec * rinv - (R)pc.A + (R)pc.B * (r - (R)pc.rc));
  const R isg = R(1) / sg;
  if (!alch) {
    dsig = S * flj * isg;
    deps = S * lj4;
    dqq = D;
    return;
  }
  if (SCHED == 0) {
    const R lv = la0, le = la1;
    const R y = (r2 * r2 * r2) * inv_s6;
    const R x = R(1) / ((R)pc.sc_alpha * (R(1) - lv) + y);
    dsig = lv * e4 * (R(2) * x - R(1)) * x * x * R(6) * y * isg * S;
    deps = lv * R(4) * (x * x - x) * S;
    dqq = le * D;
  } else {
    const R hA = la0, hB = la1;
    const R xr = r * isg;
    const R t = R(1) - xr;
    const R poly = t * (R(24) + t * (R(228) + t * (R(1232) + t * (R(-3516) + t * (R(3019.2) + t * R(-868))))));
    const R dpt = R(24) + t * (R(456) + t * (R(3696) + t * (R(-14064) + t * (R(15096) + t * R(-5208)))));
    const bool cap = xr < R(1);
    const R uc_s = cap ? R(0.25) * e4 * dpt * xr : flj;   // sigma d(eps u_cap)/dsigma
    const R uc_e = cap ? poly : lj4;                     // d(eps u_cap)/deps
    dsig = (hA * flj + hB * uc_s) * isg * S;
    deps = (hA * lj4 + hB * uc_e) * S;
    dqq = hA * D;
  }
}

template <typename R, int SCHED, bool SW>
__global__ void __launch_bounds__(kBlk) k_pgrad(Dev d, PotConsts pc, const double* __restrict__ xin,
                                                const double* __restrict__ g_energy) {
  __shared__ double acc[3 * kMaxTypes];
  __shared__ double se_t[kMaxTypes], q_t[kMaxTypes];
  const int T = d.n_types;
  for (int i = threadIdx.x; i < 3 * T; i += blockDim.x) acc[i] = 0.0;
  for (int i = threadIdx.x; i < T; i += blockDim.x) {
    se_t[i] = sqrt(d.type_eps[i]);
    q_t[i] = d.type_q[i];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int il = lane & 7, jl = lane >> 3;
  const int n_units = d.ctr[CTR_NUNIT];
  const int wave = blockIdx.x * (kBlk / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int n_waves = gridDim.x * (kBlk / 64);
  for (int u = wave; u < n_units; u += n_waves) {
    const int4 U = d.units[u];
    const int s = U.x, rep = U.w;
    const double g = g_energy[rep];
    if (g == 0.0) continue;
    const ReplicaInfo& rp = d.reps[rep];
    const double L0 = rp.box[0], L1 = rp.box[1], L2 = rp.box[2];
    const LamState lam = d.lam[rep];
    const R la0 = (R)lam.a[0], la1 = (R)lam.a[1];
    for (int e = U.y; e < U.z; ++e) {
      const int jc = d.ent_jc[e];
      const uint32_t info = d.ent_info[e];
      const uint32_t imask = info & 0xffu;
      const bool alch = ((info >> 8) & 3u) == KIND_ALCH;
      const int code = (int)((info >> 16) & 31u);
      const int sj = jc >> 3;
      const double odx = d.sc_origin[3 * sj] + (double)(code % 3 - 1) * L0 - d.sc_origin[3 * s];
      const double ody = d.sc_origin[3 * sj + 1] + (double)((code / 3) % 3 - 1) * L1 - d.sc_origin[3 * s + 1];
      const double odz = d.sc_origin[3 * sj + 2] + (double)(code / 9 - 1) * L2 - d.sc_origin[3 * s + 2];
      const int aj = max(0, d.slot_atom[jc * kCl + jl]);
      const double xj = local_x(d, xin, aj, sj, 0, L0) + odx;
      const double yj = local_x(d, xin, aj, sj, 1, L1) + ody;
      const double zj = local_x(d, xin, aj, sj, 2, L2) + odz;
      const int tj = d.atom_type[aj];
      for (int c = 0; c < kScCl; ++c) {
        if (!(imask & (1u << c))) continue;
        const bool valid = (d.ent_mask[(size_t)e * kScCl + c] >> lane) & 1ull;
        const int ai = max(0, d.slot_atom[s * kSc + c * kCl + il]);
        const R dx = (R)(xj - local_x(d, xin, ai, s, 0, L0));
        const R dy = (R)(yj - local_x(d, xin, ai, s, 1, L1));
        const R dz = (R)(zj - local_x(d, xin, ai, s, 2, L2));
        const R r2 = dx * dx + dy * dy + dz * dz;
        if (!valid || !(r2 < (R)pc.rc2)) continue;
        const int ti = d.atom_type[ai];
        const double4 tp = d.tp64[ti * T + tj];
        R dsig, deps, dqq;
        pair_param_derivs<R, SCHED, SW>(r2, alch, (R)tp.x, (R)tp.y, (R)tp.w, la0, la1, pc, dsig, deps, dqq);
        const double ws = g * 0.5 * (double)dsig, we = g * (double)deps, wq = g * (double)dqq;
        atomicAdd(&acc[ti], ws);
        atomicAdd(&acc[tj], ws);
        atomicAdd(&acc[T + ti], we * se_t[tj]);
        atomicAdd(&acc[T + tj], we * se_t[ti]);
        atomicAdd(&acc[2 * T + ti], wq * q_t[tj]);
        atomicAdd(&acc[2 * T + tj], wq * q_t[ti]);
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 3 * T; i += blockDim.x) d.pgrad_part[(size_t)blockIdx.x * 3 * T + i] = acc[i];
}

// Fixed-order sum of the block partials.
__global__ void k_pgrad_final(Dev d, int n_blocks, double* __restrict__ d_sigma, double* __restrict__ d_sqrt_eps,
                              double* __restrict__ d_charge) {
  const int T = d.n_types;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < 3 * T; i += gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int b = 0; b < n_blocks; ++b) s += d.pgrad_part[(size_t)b * 3 * T + i];
    const int which = i / T, t = i % T;
    double* out = which == 0 ? d_sigma : (which == 1 ? d_sqrt_eps : d_charge);
    if (out) out[t] = s;
  }
}

hipError_t launch_param_grads(const Dev& d, hipStream_t st, const PotConsts& pc, int precision, int schedule,
                              const double* xin, const double* g_energy, double* d_sigma, double* d_sqrt_eps,
                              double* d_charge) {
  const dim3 G(kPgBlocks), B(kBlk);
  const bool sw = pc.inv_w > 0;
#define PG(R, S, W) hipLaunchKernelGGL((k_pgrad<R, S, W>), G, B, 0, st, d, pc, xin, g_energy)
  if (precision == 0) {
    if (schedule == 0) { if (sw) PG(float, 0, true); else PG(float, 0, false); }
    else { if (sw) PG(float, 1, true); else PG(float, 1, false); }
  } else {
    if (schedule == 0) { if (sw) PG(double, 0, true); else PG(double, 0, false); }
    else { if (sw) PG(double, 1, true); else PG(double, 1, false); }
  }
#undef PG
  hipLaunchKernelGGL(k_pgrad_final, dim3(1), dim3(kBlk), 0, st, d, (int)kPgBlocks, d_sigma, d_sqrt_eps, d_charge);
  return hipGetLastError();
}

// d_pos += g_k dU/dx = -g_k F ; d_lambda = g_k dU/dlambda (last forward).
__global__ void k_backward_finish(Dev d, double inv_scale, const double* __restrict__ g_energy, double* d_pos,
                                  double* d_lambda) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (d_lambda && t < d.n_reps) d_lambda[t] = g_energy[t] * d.last_dudl[t];
  if (!d_pos) return;
  const int slots = d.sc_cap * kSc;
  for (int a = t; a < d.n_atoms; a += gridDim.x * blockDim.x) {
    const double g = g_energy[d.grids[d.atom_grid[a]].replica];
    const int sl = d.atom_slot[a];
    for (int c = 0; c < 3; ++c) d_pos[3 * a + c] -= g * (double)(long long)d.ffix[c * slots + sl] * inv_scale;
  }
}

hipError_t launch_backward_finish(const Dev& d, hipStream_t st, int precision, const double* g_energy,
                                  double* d_pos, double* d_lambda) {
  const int g = max(1, min(1024, (max(d.n_atoms, d.n_reps) + kBlk - 1) / kBlk));
  hipLaunchKernelGGL(k_backward_finish, dim3(g), dim3(kBlk), 0, st, d, 1.0 / fixed_scale(precision), g_energy,
                     d_pos, d_lambda);
  return hipGetLastError();
}

// ------------------------------------------------------------ dihedrals

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

__global__ void k_dihedrals(const double* __restrict__ pos, int n_cv, const int* __restrict__ idx,
                            double* __restrict__ xi_out, double* __restrict__ dxi, const double* __restrict__ mass_inv,
                            double* __restrict__ msum, const double* __restrict__ s, const double* __restrict__ kappa,
                            double* __restrict__ u_dafed, double* __restrict__ forces, const ReplicaInfo* reps,
                            const int* atom_rep, int n_atoms, unsigned int* flags) {
  __shared__ double dval[kBlk];
  __shared__ double ublk[kBlk];
  for (int c0 = 0; c0 < n_cv; c0 += kBlk) {
    const int c = c0 + threadIdx.x;
    double du = 0.0, d_wrap = 0.0;
    V3 g[4] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    bool ok = c < n_cv;
    int a[4] = {0, 0, 0, 0};
    if (ok) {
      for (int j = 0; j < 4; ++j) {
        a[j] = idx[4 * c + j];
        ok = ok && a[j] >= 0 && a[j] < n_atoms;
      }
      if (!ok) atomicOr(flags, 64u);  // invalid atom index: CV skipped
    }
    if (ok) {
      const ReplicaInfo& rp = reps[atom_rep[a[1]]];
      V3 r[4];
      for (int j = 0; j < 4; ++j) r[j] = {pos[3 * a[j]], pos[3 * a[j] + 1], pos[3 * a[j] + 2]};
      V3 F = sub(r[0], r[1]), G = sub(r[1], r[2]), H = sub(r[3], r[2]);
      F = {mi1(F.x, rp.box[0]), mi1(F.y, rp.box[1]), mi1(F.z, rp.box[2])};
      G = {mi1(G.x, rp.box[0]), mi1(G.y, rp.box[1]), mi1(G.z, rp.box[2])};
      H = {mi1(H.x, rp.box[0]), mi1(H.y, rp.box[1]), mi1(H.z, rp.box[2])};
      const double xi = dihedral_grad(F, G, H, g);
      xi_out[c] = xi;
      for (int j = 0; j < 4; ++j) {
        dxi[12 * c + 3 * j] = g[j].x;
        dxi[12 * c + 3 * j + 1] = g[j].y;
        dxi[12 * c + 3 * j + 2] = g[j].z;
      }
      if (mass_inv && msum) {
        double m = 0.0;
        for (int j = 0; j < 4; ++j) m += mass_inv[a[j]] * dot(g[j], g[j]);
        msum[c] = m;
      }
      if (s && kappa) {
        // periodic angular displacement wrapped into (-pi, pi]
        double dd = xi - s[c];
        dd = dd - 2.0 * M_PI * floor((dd + M_PI) / (2.0 * M_PI));
        if (dd == -M_PI) dd = M_PI;
        d_wrap = kappa[c] * dd;
        du = 0.5 * kappa[c] * dd * dd;
      }
    }
    ublk[threadIdx.x] = du;
    dval[threadIdx.x] = d_wrap;
    __syncthreads();
    if (threadIdx.x == 0 && s && kappa) {
      // fixed order: energies and forces of this chunk of CVs
      double acc = u_dafed ? (c0 == 0 ? 0.0 : u_dafed[0]) : 0.0;
      for (int k = 0; k < kBlk && c0 + k < n_cv; ++k) acc += ublk[k];
      if (u_dafed) u_dafed[0] = acc;
    }
    if (forces && s && kappa) {
      // serialize the scatter over the CVs of this chunk for a fixed order
      for (int k = 0; k < kBlk && c0 + k < n_cv; ++k) {
        if ((int)threadIdx.x == k && ok) {
          for (int j = 0; j < 4; ++j) {
            const int aj = idx[4 * c + j];
            forces[3 * aj] -= d_wrap * g[j].x;
            forces[3 * aj + 1] -= d_wrap * g[j].y;
            forces[3 * aj + 2] -= d_wrap * g[j].z;
          }
        }
        __syncthreads();
      }
    }
    __syncthreads();
  }
}

hipError_t launch_dihedrals(hipStream_t st, const double* pos, int n_cv, const int* idx, double* xi, double* dxi,
                            const double* mass_inv, double* msum, const double* s, const double* kappa,
                            double* u_dafed, double* forces, const ReplicaInfo* reps, const int* atom_rep,
                            int n_atoms, unsigned int* flags) {
  hipLaunchKernelGGL(k_dihedrals, dim3(1), dim3(kBlk), 0, st, pos, n_cv, idx, xi, dxi, mass_inv, msum, s, kappa,
                     u_dafed, forces, reps, atom_rep, n_atoms, flags);
  return hipGetLastError();
}

// ------------------------------------------------------------ lambda / OPES

// periodic Gaussian on [0, 2) (images at -2, 0, +2) and its derivative
__device__ inline void pgauss(double dth, double sig, double& v, double& dv) {
  v = dv = 0.0;
  const double inv = 1.0 / (sig * sig);
  for (int im = -1; im <= 1; ++im) {
    const double x = dth + 2.0 * im;
    const double g = exp(-0.5 * x * x * inv);
    v += g;
    dv += -x * inv * g;
  }
}

// Block-wide sums over the kernel centres at theta: weighted (Standard) and
// unweighted (Explore) density and their theta derivatives.  Fixed order.
__device__ void kde_sums(const double* cen, const double* w, int n, double th, double sig, double out[4]) {
  __shared__ double red[4][kBlk];
  double a[4] = {0, 0, 0, 0};
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    double v, dv;
    pgauss(th - cen[j], sig, v, dv);
    a[0] += w[j] * v;
    a[1] += w[j] * dv;
    a[2] += v;
    a[3] += dv;
  }
  for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = a[k];
  __syncthreads();
  for (int off = kBlk / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off)
      for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + off];
    __syncthreads();
  }
  for (int k = 0; k < 4; ++k) out[k] = red[k][0];
  __syncthreads();
}

// U_total and dU/dtheta from the sums (eq. 11 for each bias, eq. 14 total).
__device__ inline void opes_bias(const double* h, const double sums[4], double& U, double& dU) {
  const double n = h[OPES_N];
  U = dU = 0.0;
  if (n < 1.0) return;
  const double kT = h[OPES_KT];
  const double gs = h[OPES_DE_STD] / kT, ge = h[OPES_DE_EXPL] / kT;
  const double nus = 1.0 - 1.0 / gs, nue = ge - 1.0;
  const double es = exp(-gs / nus), ee = exp(-ge / nue);
  // rho_hat / rho_bar = (A / W) / (S / (n W)) = n A / S
  const double rs = n * sums[0] / h[OPES_S_STD], re = n * sums[2] / h[OPES_S_EXPL];
  const double drs = n * sums[1] / h[OPES_S_STD], dre = n * sums[3] / h[OPES_S_EXPL];
  U = nus * kT * log(rs + es) + nue * kT * log(re + ee);
  dU = nus * kT * drs / (rs + es) + nue * kT * dre / (re + ee);
}

__global__ void __launch_bounds__(kBlk) k_opes(double* __restrict__ st, const double* __restrict__ dudl,
                                               double* __restrict__ lam_out, int deposit) {
  double* h = st;
  const int cap = (int)h[OPES_CAP];
  double* grid_u = st + OPES_HEADER;
  double* grid_du = grid_u + OPES_GRID_N;
  double* cen = grid_du + OPES_GRID_N;
  double* w = cen + cap;
  const double sig = h[OPES_SIGMA];
  double th = h[OPES_THETA];
  th = th - 2.0 * floor(th / 2.0);
  if (th >= 2.0) th = 0.0;
  __shared__ double sh_n;
  if (threadIdx.x == 0) sh_n = h[OPES_N];
  __syncthreads();
  int n = (int)sh_n;
  double sums[4];
  if (deposit && n < cap) {
    kde_sums(cen, w, n, th, sig, sums);
    double U, dU;
    opes_bias(h, sums, U, dU);
    const double wn = exp(U / h[OPES_KT]);
    if (threadIdx.x == 0) {
      double g0, dg0;
      pgauss(0.0, sig, g0, dg0);
      // pair sums over centres gain the new row, the new column and the diagonal
      h[OPES_S_STD] += sums[0] + wn * sums[2] + wn * g0;
      h[OPES_S_EXPL] += 2.0 * sums[2] + g0;
      h[OPES_W_STD] += wn;
      cen[n] = th;
      w[n] = wn;
      h[OPES_N] = (double)(n + 1);
    }
    __syncthreads();
    n = n + 1;
  }
  kde_sums(cen, w, n, th, sig, sums);
  double U, dU;
  opes_bias(h, sums, U, dU);
  if (threadIdx.x == 0) {
    const double lam = th <= 1.0 ? th : 2.0 - th;
    const double dl = th <= 1.0 ? 1.0 : -1.0;
    h[OPES_THETA] = th;
    h[OPES_LAMBDA] = lam;
    h[OPES_DLAM] = dl;
    h[OPES_U] = U;
    h[OPES_DU] = dU;
    h[OPES_FTHETA] = -dl * (dudl ? dudl[0] : 0.0) - dU;
    if (lam_out) lam_out[0] = lam;
  }
  if (deposit) {
    // bias on the output grid (diagnostics), one node at a time
    for (int g = 0; g < OPES_GRID_N; ++g) {
      const double tg = 2.0 * g / OPES_GRID_N;
      kde_sums(cen, w, n, tg, sig, sums);
      double Ug, dUg;
      opes_bias(h, sums, Ug, dUg);
      if (threadIdx.x == 0) {
        grid_u[g] = Ug;
        grid_du[g] = dUg;
      }
    }
  }
}

__global__ void k_opes_init(double* st, int cap, double kT, double sigma, double de_std, double de_expl,
                            double theta0) {
  const int total = OPES_HEADER + 2 * OPES_GRID_N + 2 * cap;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) st[i] = 0.0;
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st[OPES_THETA] = theta0;
    st[OPES_KT] = kT;
    st[OPES_SIGMA] = sigma;
    st[OPES_DE_STD] = de_std;
    st[OPES_DE_EXPL] = de_expl;
    st[OPES_CAP] = (double)cap;
  }
}

hipError_t launch_opes_init(hipStream_t st, double* state, int cap, double kT, double sigma, double de_std,
                            double de_expl, double theta0) {
  hipLaunchKernelGGL(k_opes_init, dim3(1), dim3(kBlk), 0, st, state, cap, kT, sigma, de_std, de_expl, theta0);
  return hipGetLastError();
}

hipError_t launch_opes(hipStream_t st, double* state, const double* dudl, double* lambda_out, int deposit) {
  hipLaunchKernelGGL(k_opes, dim3(1), dim3(kBlk), 0, st, state, dudl, lambda_out, deposit);
  return hipGetLastError();
}

}  // namespace anb
