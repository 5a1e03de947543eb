// Backward pass, dihedral collective variables and the lambda/OPES update.
//
// - k_pgrad: a second pass over the list (the work units of the last
//   forward, its FP64 slot coordinates and image offsets) that sums the
//   derivatives of the pair energies with respect to sigma, sqrt(epsilon)
//   and the charge, weighted by the upstream gradient of each box, per atom:
//   in registers over a unit (i-atoms) or an entry (j-atom), then as 64-bit
//   fixed-point atomics per slot, so the sums do not depend on the order of
//   the adds.  k_pgrad_final adds the slots of each atom type in a fixed
//   order (and clears them for the next pass).
// - k_backward_finish: -g_k F and g_k dU/dlambda from the last forward.
// - k_dihedrals: dihedral angles, their Cartesian gradients, the paper's
//   eq. 16 sum and the d-AFED coupling (eq. 15), one block (dihedral_cv.h).
// - k_opes: mirror-periodic theta (eq. 3), dual OPES bias (eqs. 11-14),
//   kernel deposition, generalized force on theta.  FP64, one block;
//   k_opes_grid refreshes the bias on the output grid after a deposition.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "anb_internal.h"
#include "anb_kernels.h"
#include "dihedral_cv.h"
#include "erfc_coeffs.h"
#include "lane_ops.h"
#include "pair_math.h"

namespace anb {

constexpr int kBlk = 256;
constexpr int kPgBlocks = 1024;   // blocks of the parameter-gradient pass (4 waves per SIMD)
constexpr int kPgLdsTypes = 32;   // the type-pair table goes to LDS up to this many types

__device__ inline float rcp_(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double rcp_(double x) { return 1.0 / x; }
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
  erfc_exp((R)pc.alpha * r, ec, ex);
  const R D = (R)kKe * (ec * rinv - (R)pc.A + (R)pc.B * (r - (R)pc.rc));
  const R isg = rcp_(sg);
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

__device__ inline void pg_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// sum over the 8 lanes that differ only in the lane-index bits m0, m1, m2
// (a butterfly: the same tree, and so the same result, in every lane)
template <typename V>
__device__ inline V lane_sum(V v, int m0, int m1, int m2) {
  v += __shfl_xor(v, m0);
  v += __shfl_xor(v, m1);
  v += __shfl_xor(v, m2);
  return v;
}

// v * scale rounded into a 64-bit fixed-point slot sum
__device__ inline void add_fixed(unsigned long long* p, double v, double scale, unsigned int* flags) {
  const double x = v * scale;
  if (!(fabs(x) < 0x1p62)) {
    atomicOr(flags, 1u);
    return;
  }
  const long long iv = __double2ll_rn(x);
  if (iv != 0) atomicAdd(p, (unsigned long long)iv);
}

// One wave per work unit (grid-stride over the units): lane (jl, il) as in
// the tile kernel.  i-atom sums stay in registers for the whole unit (one
// super-cluster), j-atom sums for one entry.
template <typename R, int SCHED, bool SW>
__global__ void __launch_bounds__(kBlk) k_pgrad(Dev d, PotConsts pc, const double* __restrict__ g_energy,
                                                double scale) {
  using TP = typename std::conditional<sizeof(R) == 4, float4, double4>::type;
  __shared__ double se_t[kMaxTypes], q_t[kMaxTypes];
  // the type-pair table (rounded to the pair precision) in LDS when it fits
  // (T <= 32), else read from HBM
  __shared__ TP tp_s[kPgLdsTypes * kPgLdsTypes];
  // the current super-cluster's slots and the current unit's j-clusters
  // (image offset added; lane (k, t): atom t of entry k), one copy per wave
  __shared__ double4 ip_all[kBlk], jp_all[kBlk];
  __shared__ int it_all[kBlk], jt_all[kBlk], js_all[kBlk];
  const int T = d.n_types;
  const bool tp_lds = T <= kPgLdsTypes;
  const TP* __restrict__ tpg = reinterpret_cast<const TP*>(sizeof(R) == 4 ? (const void*)d.tp32 : (const void*)d.tp64);
  for (int i = threadIdx.x; i < T; i += kBlk) {
    se_t[i] = sqrt(d.type_eps[i]);
    q_t[i] = d.type_q[i];
  }
  if (tp_lds)
    for (int i = threadIdx.x; i < T * T; i += kBlk) tp_s[i] = tpg[i];
  __syncthreads();
  const TP* __restrict__ tpt = tp_lds ? tp_s : tpg;
  double4* ip_s = ip_all + (threadIdx.x & ~63);
  int* it_s = it_all + (threadIdx.x & ~63);
  double4* jp_s = jp_all + (threadIdx.x & ~63);
  int* jt_s = jt_all + (threadIdx.x & ~63);
  int* js_s = js_all + (threadIdx.x & ~63);
  const int lane = threadIdx.x & 63;
  const int il = lane & 7, jl = lane >> 3;
  const int slots = d.sc_cap * kSc;
  unsigned long long* acc0 = d.pg_fix;
  unsigned long long* acc1 = d.pg_fix + slots;
  unsigned long long* acc2 = d.pg_fix + 2 * (size_t)slots;
  const int n_units = d.ctr[CTR_NUNIT];
  const int wave = blockIdx.x * (kBlk / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int n_waves = gridDim.x * (kBlk / 64);
  for (int u = wave; u < n_units; u += n_waves) {
    const int4 U = d.units[u];
    const int s = U.x, rep = unit_rep(U.w);
    const double g = g_energy[rep];
    if (g == 0.0) continue;
    const LamState lam = d.lam[rep];
    const R la0 = (R)lam.a[0], la1 = (R)lam.a[1];
    {
      static_assert(kMaxEpu * kCl == 64, "one lane per atom of a unit's entries");
      const int k = lane >> 3, t = lane & 7, e = U.y + k;
      double4 v = make_double4(0.0, 0.0, 0.0, 0.0);
      int ty = 0, jsl = 0;
      const double4 pi = d.pos64[s * kSc + lane];
      const int ti = d.slot_type[s * kSc + lane];
      if (e < U.z) {
        jsl = d.ent_jc[e] * kCl + t;
        const double4 off = d.ent_off[e];
        const double4 p = d.pos64[jsl];
        v = make_double4(p.x + off.x, p.y + off.y, p.z + off.z, 0.0);
        ty = d.slot_type[jsl];
      }
      pg_wave_sync();
      ip_s[lane] = pi;
      it_s[lane] = ti;
      jp_s[lane] = v;
      jt_s[lane] = ty;
      js_s[lane] = jsl;
      pg_wave_sync();
    }
    // sums in the pair precision over one unit (i) or entry (j), then FP64
    R ai0[kScCl], ai1[kScCl], ai2[kScCl];
#pragma unroll
    for (int c = 0; c < kScCl; ++c) ai0[c] = ai1[c] = ai2[c] = R(0);
    // entry words and pair masks are read one entry ahead (scalar loads)
    uint32_t info_n = d.ent_info[U.y];
    unsigned long long m_n[kScCl];
#pragma unroll
    for (int c = 0; c < kScCl; ++c) m_n[c] = d.ent_mask[(size_t)U.y * kScCl + c];
    for (int e = U.y; e < U.z; ++e) {
      const uint32_t info = info_n;
      unsigned long long m[kScCl];
#pragma unroll
      for (int c = 0; c < kScCl; ++c) m[c] = m_n[c];
      if (e + 1 < U.z) {
        info_n = d.ent_info[e + 1];
#pragma unroll
        for (int c = 0; c < kScCl; ++c) m_n[c] = d.ent_mask[(size_t)(e + 1) * kScCl + c];
      }
      const uint32_t imask = info & 0xffu;
      const bool alch = ((info >> 8) & 3u) == KIND_ALCH;
      const int kj = (e - U.y) * kCl + jl;
      const int jsl = js_s[kj];
      const double4 pj = jp_s[kj];
      const double xj = pj.x, yj = pj.y, zj = pj.z;
      const int tj = jt_s[kj];
      const R sej = (R)se_t[tj], qj = (R)q_t[tj];
      R bj0 = R(0), bj1 = R(0), bj2 = R(0);
#pragma unroll
      for (int c = 0; c < kScCl; ++c) {
        if (!(imask & (1u << c))) continue;
        const double4 pi = ip_s[c * kCl + il];
        const R dx = (R)(xj - pi.x), dy = (R)(yj - pi.y), dz = (R)(zj - pi.z);
        const R r2 = dx * dx + dy * dy + dz * dz;
        const bool valid = ((m[c] >> lane) & 1ull) && r2 < (R)pc.rc2;
        if (__ballot(valid) == 0) continue;
        const int ti = it_s[c * kCl + il];
        const TP tp = tpt[ti * T + tj];
        R dsig, deps, dqq;
        pair_param_derivs<R, SCHED, SW>(valid ? r2 : R(1), alch, (R)tp.x, (R)tp.y, (R)tp.w, la0, la1, pc, dsig,
                                        deps, dqq);
        const R ws = valid ? R(0.5) * dsig : R(0);
        const R we = valid ? deps : R(0);
        const R wq = valid ? dqq : R(0);
        ai0[c] += ws;
        ai1[c] += we * sej;
        ai2[c] += wq * qj;
        bj0 += ws;
        bj1 += we * (R)se_t[ti];
        bj2 += wq * (R)q_t[ti];
      }
      // the j-atom's sums over il, weighted by the box's upstream gradient
      const double vj0 = g * (double)red8(bj0);
      const double vj1 = g * (double)red8(bj1);
      const double vj2 = g * (double)red8(bj2);
      if (il == 0) {
        add_fixed(acc0 + jsl, vj0, scale, d.flags);
        add_fixed(acc1 + jsl, vj1, scale, d.flags);
        add_fixed(acc2 + jsl, vj2, scale, d.flags);
      }
    }
    // the i-atoms' sums over jl, reduce-scattered so that lane l holds slot
    // s * 64 + l (one atomic per lane and component)
    {
      const bool odd8 = (lane & 8) != 0;
      const R v0 = scatter_jl(ai0, odd8), v1 = scatter_jl(ai1, odd8), v2 = scatter_jl(ai2, odd8);
      const int isl = s * kSc + lane;
      add_fixed(acc0 + isl, g * (double)v0, scale, d.flags);
      add_fixed(acc1 + isl, g * (double)v1, scale, d.flags);
      add_fixed(acc2 + isl, g * (double)v2, scale, d.flags);
    }
  }
}

// Block (component, type): the slot sums of that type's atoms, each thread
// over a fixed stride of slots, then the waves' butterflies and the waves in
// order; the slots it read are cleared for the next pass.
constexpr int kPgFinalBlk = 1024;
constexpr int kPgFinalRun = 16;
__global__ void __launch_bounds__(kPgFinalBlk) k_pgrad_final(Dev d, double inv_scale, double* __restrict__ d_sigma,
                                                             double* __restrict__ d_sqrt_eps,
                                                             double* __restrict__ d_charge,
                                                             double* __restrict__ d_eps) {
  __shared__ double part[kPgFinalBlk / 64];
  const int T = d.n_types;
  const int comp = blockIdx.x / T, t = blockIdx.x % T;
  const int slots = d.sc_cap * kSc;
  unsigned long long* acc = d.pg_fix + (size_t)comp * slots;
  double sum = 0.0;
  // kPgFinalRun slots per thread per round, all loads of a round issued
  // together (padding slots carry type 0 and zero sums)
  for (int base = 0; base < slots; base += kPgFinalBlk * kPgFinalRun) {
    int ty[kPgFinalRun];
    long long v[kPgFinalRun];
#pragma unroll
    for (int i = 0; i < kPgFinalRun; ++i) {
      const int sl = base + i * kPgFinalBlk + threadIdx.x;
      ty[i] = sl < slots ? d.slot_type[sl] : -1;
      v[i] = sl < slots ? (long long)acc[sl] : 0ll;
    }
#pragma unroll
    for (int i = 0; i < kPgFinalRun; ++i) {
      if (ty[i] != t || v[i] == 0) continue;
      sum += (double)v[i] * inv_scale;
      acc[base + i * kPgFinalBlk + threadIdx.x] = 0ull;
    }
  }
  sum = lane_sum(sum, 1, 2, 4);
  sum = lane_sum(sum, 8, 16, 32);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    double total = 0.0;
    for (int w = 0; w < kPgFinalBlk / 64; ++w) total += part[w];
    double* out = comp == 0 ? d_sigma : (comp == 1 ? d_sqrt_eps : d_charge);
    if (out) out[t] = total;
    // eps_ij = sqrt(eps_i) sqrt(eps_j): dU/deps_t = dU/dsqrt(eps_t) / (2 sqrt(eps_t)), which has no
    // value where eps_t = 0 (NaN there)
    if (comp == 1 && d_eps) {
      const double e = d.type_eps[t];
      d_eps[t] = e > 0.0 ? total / (2.0 * sqrt(e)) : __builtin_nan("");
    }
  }
}

hipError_t launch_param_grads(const Dev& d, hipStream_t st, const PotConsts& pc, int precision, int schedule,
                              const double* g_energy, double* d_sigma, double* d_sqrt_eps, double* d_charge,
                              double* d_eps) {
  const dim3 G(kPgBlocks), B(kBlk);
  const bool sw = pc.inv_w > 0;
  const double scale = fixed_scale(precision);
#define PG(R, S, W) hipLaunchKernelGGL((k_pgrad<R, S, W>), G, B, 0, st, d, pc, g_energy, scale)
  if (precision == 0) {
    if (schedule == 0) { if (sw) PG(float, 0, true); else PG(float, 0, false); }
    else { if (sw) PG(float, 1, true); else PG(float, 1, false); }
  } else {
    if (schedule == 0) { if (sw) PG(double, 0, true); else PG(double, 0, false); }
    else { if (sw) PG(double, 1, true); else PG(double, 1, false); }
  }
#undef PG
  hipLaunchKernelGGL(k_pgrad_final, dim3(3 * d.n_types), dim3(kPgFinalBlk), 0, st, d, 1.0 / scale, d_sigma, d_sqrt_eps,
                     d_charge, d_eps);
  return hipGetLastError();
}

// d_pos += g_k dU/dx = -g_k F ; d_lambda = g_k dU/dlambda (last forward).
__global__ void k_backward_finish(Dev d, double inv_scale, const double* __restrict__ g_energy, double* d_pos,
                                  double* d_lambda) {
  const int t = blockIdx.x * kBlk + threadIdx.x;
  if (d_lambda && t < d.n_reps) d_lambda[t] = g_energy[t] * d.last_dudl[t];
  if (!d_pos) return;
  const int slots = d.sc_cap * kSc;
  for (int a = t; a < d.n_atoms; a += gridDim.x * kBlk) {
    const double g = g_energy[d.atom_rep[a]];
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

__global__ void __launch_bounds__(kBlk) k_dihedrals(const double* __restrict__ pos, int n_cv,
                                                    const int* __restrict__ idx, double* __restrict__ xi_out,
                                                    double* __restrict__ dxi, const double* __restrict__ mass_inv,
                                                    double* __restrict__ msum, const double* __restrict__ s,
                                                    const double* __restrict__ kappa, double* __restrict__ u_dafed,
                                                    double* __restrict__ forces, const ReplicaInfo* reps,
                                                    const int* atom_rep, int n_atoms, unsigned int* flags) {
  const dcv::CvOut o{xi_out, dxi, mass_inv, msum, u_dafed, forces};
  dcv::cv_block<kBlk>(pos, n_cv, idx, s, kappa, o, reps, atom_rep, n_atoms, flags, [](int, bool, double) {});
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
  __shared__ double red[4][kBlk / 64];
  double a[4] = {0, 0, 0, 0};
  for (int j = threadIdx.x; j < n; j += kBlk) {
    double v, dv;
    pgauss(th - cen[j], sig, v, dv);
    a[0] += w[j] * v;
    a[1] += w[j] * dv;
    a[2] += v;
    a[3] += dv;
  }
  // butterflies within each wave, then the waves in order (the same order
  // in every thread)
  for (int k = 0; k < 4; ++k) {
    a[k] = lane_sum(a[k], 1, 2, 4);
    a[k] = lane_sum(a[k], 8, 16, 32);
  }
  if ((threadIdx.x & 63) == 0)
    for (int k = 0; k < 4; ++k) red[k][threadIdx.x >> 6] = a[k];
  __syncthreads();
  for (int k = 0; k < 4; ++k) {
    double t = red[k][0];
    for (int q = 1; q < kBlk / 64; ++q) t += red[k][q];
    out[k] = t;
  }
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
}

// The bias on the output grid (diagnostics) after a deposition: block g
// takes node g.
__global__ void __launch_bounds__(kBlk) k_opes_grid(double* __restrict__ st) {
  const double* h = st;
  const int cap = (int)h[OPES_CAP];
  double* grid_u = st + OPES_HEADER;
  double* grid_du = grid_u + OPES_GRID_N;
  const double* cen = grid_du + OPES_GRID_N;
  const double* w = cen + cap;
  const int g = blockIdx.x;
  double sums[4];
  kde_sums(cen, w, (int)h[OPES_N], 2.0 * g / OPES_GRID_N, h[OPES_SIGMA], sums);
  double Ug, dUg;
  opes_bias(h, sums, Ug, dUg);
  if (threadIdx.x == 0) {
    grid_u[g] = Ug;
    grid_du[g] = dUg;
  }
}

__global__ void k_opes_init(double* st, int cap, double kT, double sigma, double de_std, double de_expl,
                            double theta0) {
  const int total = OPES_HEADER + 2 * OPES_GRID_N + 2 * cap;
  for (int i = blockIdx.x * kBlk + threadIdx.x; i < total; i += gridDim.x * kBlk) st[i] = 0.0;
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
  if (deposit) hipLaunchKernelGGL(k_opes_grid, dim3(OPES_GRID_N), dim3(kBlk), 0, st, state);
  return hipGetLastError();
}

}  // namespace anb
