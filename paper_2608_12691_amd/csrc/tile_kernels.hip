// Per-call kernels: lambda factors and displacement check, canonical local
// coordinates, the cluster-pair tile kernel, and the final reductions.
//
// Tile kernel layout (one wave = one work unit = one i-super-cluster and a
// run of its list entries):
//   lane = jl * 8 + il: il is the i-atom inside an i-cluster, jl the atom of
//   the entry's j-cluster.  The 8 i-clusters of the super-cluster are held
//   in registers for the whole unit; for each entry the wave loads one
//   j-cluster (8 atoms, each read by 8 lanes) and loops over the i-clusters
//   its mask selects, so one pass covers up to 8 x 64 atom pairs.
//   j-forces are summed over the 8 i-clusters in registers and then over il
//   with DPP lane moves, and leave with one 64-bit fixed-point atomic per
//   component and j-atom; i-forces stay in registers until the unit ends.
// Pair arithmetic is FP32 (or FP64 in the reference path); positions are
// super-cluster-local so that FP32 keeps ~1e-7 A resolution in any box.
#include <hip/hip_runtime.h>

#include "anb_internal.h"
#include "anb_kernels.h"
#include "erfc_coeffs.h"

namespace anb {

constexpr int kBlk = 256;

__device__ inline int gtid() { return blockIdx.x * blockDim.x + threadIdx.x; }
__device__ inline int gthreads() { return gridDim.x * blockDim.x; }

// ------------------------------------------------------------ math by type

__device__ inline float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ inline double rsq(double x) { return 1.0 / sqrt(x); }
__device__ inline float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double rcp(double x) { return 1.0 / x; }
__device__ inline float clamp01(float x) { return __builtin_amdgcn_fmed3f(x, 0.0f, 1.0f); }
__device__ inline double clamp01(double x) { return fmin(fmax(x, 0.0), 1.0); }

// erfc(x) and exp(-x^2) for 0 <= x <= ANB_ERFC_XMAX
__device__ inline void erfc_exp(float x, float& ec, float& ex) {
  const float t = __builtin_amdgcn_rcpf(fmaf(ANB_ERFC_P, x, 1.0f));
  float p = kErfcCoef[ANB_ERFC_DEG];
#pragma unroll
  for (int k = ANB_ERFC_DEG - 1; k >= 0; --k) p = fmaf(p, t, kErfcCoef[k]);
  ex = __builtin_amdgcn_exp2f((x * x) * -1.4426950408889634f);
  ec = t * p * ex;
}
__device__ inline void erfc_exp(double x, double& ec, double& ex) {
  ex = exp(-x * x);
  ec = erfc(x);
}

template <typename R>
struct C4 {};
template <>
struct C4<float> {
  using P4 = float4;
  using P2 = float2;
};
template <>
struct C4<double> {
  using P4 = double4;
  using P2 = double2;
};

template <typename R>
struct Pot {
  R rc2, rc, rs, inv_w, alpha, A, B, c2a, sca;
};

template <typename R>
__host__ Pot<R> make_pot(const PotConsts& p) {
  Pot<R> o;
  o.rc2 = (R)p.rc2;
  o.rc = (R)p.rc;
  o.rs = (R)p.rs;
  o.inv_w = (R)p.inv_w;
  o.alpha = (R)p.alpha;
  o.A = (R)p.A;
  o.B = (R)p.B;
  o.c2a = (R)p.c2a;
  o.sca = (R)p.sc_alpha;
  return o;
}

// Switched LJ, DSF and the scalar pair force.  All lanes compute; lanes
// outside the cutoff or masked out get r2 := 1 so every value stays finite,
// and their outputs are selected to zero.
template <typename R, bool SW>
struct PairCore {
  R r2s, rinv, rinv2, r;
  R lj0, flj0;   // unswitched LJ and -r dLJ/dr
  R S, rdS;      // switch and r dS/dr
  R el, fel;     // q q D(r) and -r d(q q D)/dr
  __device__ inline void eval(R r2, bool inr, R sij, R e4, R qq, const Pot<R>& P) {
    r2s = inr ? r2 : R(1);
    rinv = rsq(r2s);
    rinv2 = rinv * rinv;
    r = r2s * rinv;
    const R s2 = sij * sij * rinv2;
    const R s6 = s2 * s2 * s2;
    lj0 = e4 * s6 * (s6 - R(1));
    flj0 = e4 * s6 * (R(12) * s6 - R(6));
    if (SW) {
      const R t = clamp01((r - P.rs) * P.inv_w);
      const R t2 = t * t;
      S = R(1) - t2 * t * (R(10) + t * (R(-15) + R(6) * t));
      const R omt = R(1) - t;
      rdS = R(-30) * t2 * omt * omt * P.inv_w * r;
    } else {
      S = R(1);
      rdS = R(0);
    }
    R ec, ex;
    erfc_exp(P.alpha * r, ec, ex);
    const R erinv = ec * rinv;
    el = qq * (erinv - P.A + P.B * (r - P.rc));
    fel = qq * (erinv + P.c2a * ex - P.B * r);
  }
};

// ------------------------------------------------------------ DPP helpers

// sum over the 8 lanes of each lane group (lane & ~7): quad_perm xor 1, xor 2, row_half_mirror
__device__ inline float red8(float v) {
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, false));
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x141, 0xF, 0xF, false));
  return v;
}
__device__ inline double dpp_d(double v, int ctrl) {
  const long long b = __double_as_longlong(v);
  int lo = (int)(b & 0xffffffffll), hi = (int)(b >> 32);
  if (ctrl == 0xB1) {
    lo = __builtin_amdgcn_mov_dpp(lo, 0xB1, 0xF, 0xF, false);
    hi = __builtin_amdgcn_mov_dpp(hi, 0xB1, 0xF, 0xF, false);
  } else if (ctrl == 0x4E) {
    lo = __builtin_amdgcn_mov_dpp(lo, 0x4E, 0xF, 0xF, false);
    hi = __builtin_amdgcn_mov_dpp(hi, 0x4E, 0xF, 0xF, false);
  } else {
    lo = __builtin_amdgcn_mov_dpp(lo, 0x141, 0xF, 0xF, false);
    hi = __builtin_amdgcn_mov_dpp(hi, 0x141, 0xF, 0xF, false);
  }
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ inline double red8(double v) {
  v += dpp_d(v, 0xB1);
  v += dpp_d(v, 0x4E);
  v += dpp_d(v, 0x141);
  return v;
}
// sum over lanes with equal (lane & 7): xor 8, 16, 32
template <typename R>
__device__ inline R red_jl(R v) {
  v += __shfl_xor(v, 8);
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  return v;
}
__device__ inline double wave_sum(double v) {
  for (int o = 1; o < 64; o <<= 1) v += __shfl_xor(v, o);
  return v;
}

// Read-only view of list data inside the tile kernel: the constant address
// space tells the compiler the memory is not written during the launch, so
// wave-uniform reads become scalar loads.
template <typename T>
using cptr = const __attribute__((address_space(4))) T*;
template <typename T>
__device__ inline cptr<T> as_const(const T* p) {
  return (cptr<T>)p;
}

// Orders this wave's LDS writes before other lanes of the same wave read
// them (each wave owns its LDS slice, so no block-wide barrier is needed).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename R>
__device__ inline void add_fixed(unsigned long long* p, R v, double scale, unsigned int* flags) {
  if (v == R(0)) return;
  const double x = (double)v * scale;
  if (!(fabs(x) < 4.611686018427388e18)) {  // |f| >= 2^62 / scale, or NaN
    atomicOr(flags, 1u);
    return;
  }
  atomicAdd(p, (unsigned long long)__double2ll_rn(x));
}

// ------------------------------------------------------------ tile kernel

// Coordinate k of atom a relative to the origin of its super-cluster s, in
// the periodic image the atom had when the list was built: the displacement
// since the build (minimum image) plus the build-time wrapped offset.  This
// stays consistent with the list's image shifts for any super-cluster extent.
__device__ inline double local_coord(const Dev& d, const double* __restrict__ x, int a, int s, int k, double L) {
  double m = x[3 * a + k] - d.x_build[3 * a + k];
  m -= L * rint(m / L);
  return m + (d.xw[3 * a + k] - d.sc_origin[3 * s + k]);
}

// Solute-solvent pair (rare: only entries of kind KIND_ALCH).  Its inputs
// are taken from FP64 sources and rounded once: the displacement from the
// FP64 positions (minimum image), and sigma_ij, 4 eps_ij, k_e q_i q_j and
// 1/sigma_ij^6 from a per-type-pair table built in FP64.  This keeps the
// lambda derivative, a sum with cancellation, at FP32 rounding level.
template <typename R, int SCHED, bool SW>
__device__ inline void alch_pair(R dx, R dy, R dz, bool valid, const typename C4<R>::P4& tp, R lv_or_hA, R le_or_hB,
                                 const Pot<R>& P, R& u, R& fr, R& rinv2, bool& inr, double& a0, double& a1,
                                 double& a2) {
  const R r2 = dx * dx + dy * dy + dz * dz;
  inr = valid && r2 < P.rc2;
  const R sij = tp.x, e4 = tp.y, qq = tp.z, inv_s6 = tp.w;
  PairCore<R, SW> pc;
  pc.eval(r2, inr, sij, e4, qq, P);
  rinv2 = pc.rinv2;
  if (SCHED == 0) {
    // Beutler soft core: lv 4eps (x^2 - x) S + le qq D
    const R lv = lv_or_hA, le = le_or_hB;
    const R y = (pc.r2s * pc.r2s * pc.r2s) * inv_s6;
    const R x = rcp(P.sca * (R(1) - lv) + y);
    const R core = e4 * (x * x - x);
    const R dcx = e4 * (R(2) * x - R(1));
    const R uv = lv * core * pc.S;
    const R fv = lv * (dcx * x * x * R(6) * y * pc.S - core * pc.rdS);
    const R dl = (core + lv * dcx * P.sca * x * x) * pc.S;
    u = uv + le * pc.el;
    fr = fv + le * pc.fel;
    if (inr) {
      a0 += (double)uv;
      a1 += (double)pc.el;
      a2 += (double)dl;
    }
  } else {
    // LBF: hA [LJ S + qq D] + hB eps u_cap(r/sig) S
    const R hA = lv_or_hA, hB = le_or_hB;
    const R vdw = pc.lj0 * pc.S;
    const R fvdw = pc.flj0 * pc.S - pc.lj0 * pc.rdS;
    // u_cap of eq. 6 for x < 1, written as the same polynomial expanded about
    // x = 1 (t = 1 - x), which avoids the cancellation of the monomial form
    // near the join: u = t(24 + t(228 + t(1232 + t(-3516 + t(3019.2 - 868 t)))))
    const R xr = pc.r * rcp(sij);
    const R t = R(1) - xr;
    const R epsq = R(0.25) * e4;
    const R poly = t * (R(24) + t * (R(228) + t * (R(1232) + t * (R(-3516) + t * (R(3019.2) + t * R(-868))))));
    const R dpoly_dt = R(24) + t * (R(456) + t * (R(3696) + t * (R(-14064) + t * (R(15096) + t * R(-5208)))));
    const bool cap = xr < R(1);
    const R uc = cap ? epsq * poly : pc.lj0;
    const R fuc = cap ? epsq * dpoly_dt * xr : pc.flj0;   // -r du/dr = x du/dt
    const R ubv = uc * pc.S;
    const R fub = fuc * pc.S - uc * pc.rdS;
    u = hA * (vdw + pc.el) + hB * ubv;
    fr = hA * (fvdw + pc.fel) + hB * fub;
    if (inr) {
      a0 += (double)vdw;
      a1 += (double)pc.el;
      a2 += (double)ubv;
    }
  }
}

template <typename R, int SCHED, bool SW>
__global__ void __launch_bounds__(kBlk) k_tile(Dev d, Pot<R> P, int xcd, double fscale, const double* __restrict__ xin) {
  using P4 = typename C4<R>::P4;
  using P2 = typename C4<R>::P2;
  const P4* __restrict__ pos = reinterpret_cast<const P4*>(sizeof(R) == 4 ? (const void*)d.pos32 : (const void*)d.pos64);
  const P2* __restrict__ se = reinterpret_cast<const P2*>(sizeof(R) == 4 ? (const void*)d.se32 : (const void*)d.se64);
  const P4* __restrict__ tpair = reinterpret_cast<const P4*>(sizeof(R) == 4 ? (const void*)d.tp32 : (const void*)d.tp64);
  const int slots = d.sc_cap * kSc;
  const int T = d.n_types;
  const int lane = threadIdx.x & 63;
  __shared__ P4 ipos_all[kBlk];
  __shared__ P2 ise_all[kBlk];
  P4* ipos = ipos_all + (threadIdx.x & ~63);
  P2* ise = ise_all + (threadIdx.x & ~63);
  const int il = lane & 7, jl = lane >> 3;
  const int n_units = d.ctr[CTR_NUNIT];
  // Unit range of this wave.  XCD-aware: blocks are dispatched round-robin
  // over the 8 XCDs, so XCD x (blocks b with b % 8 == x) takes the x-th
  // contiguous eighth of the units (neighbouring super-clusters share
  // j-clusters, which then stay in that XCD's L2) and splits it evenly
  // over its waves.  Otherwise consecutive waves take consecutive runs.
  // wave index made provably uniform: unit and entry indices then live in
  // scalar registers and their loads are scalar loads
  const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int ub, ue;
  if (xcd && (gridDim.x & 7) == 0) {
    const int x = blockIdx.x & 7, nbx = gridDim.x >> 3, lb = blockIdx.x >> 3;
    const int c0 = (int)((long long)n_units * x / 8), c1 = (int)((long long)n_units * (x + 1) / 8);
    const int nwx = nbx * (kBlk / 64), w = lb * (kBlk / 64) + wib;
    ub = c0 + (int)((long long)(c1 - c0) * w / nwx);
    ue = c0 + (int)((long long)(c1 - c0) * (w + 1) / nwx);
  } else {
    const int nw = gridDim.x * (kBlk / 64), w = blockIdx.x * (kBlk / 64) + wib;
    ub = (int)((long long)n_units * w / nw);
    ue = (int)((long long)n_units * (w + 1) / nw);
  }
  for (int u = ub; u < ue; ++u) {
    const cptr<int> up = as_const(reinterpret_cast<const int*>(d.units)) + 4 * u;
    const int4 U = make_int4(up[0], up[1], up[2], up[3]);
    const int s = U.x;
    const ReplicaInfo& rp = d.reps[U.w];
    const double L0 = rp.box[0], L1 = rp.box[1], L2 = rp.box[2];
    const LamState lam = d.lam[U.w];
    R la0, la1;
    if (sizeof(R) == 4) {
      la0 = (R)lam.f[0];
      la1 = (R)lam.f[1];
    } else {
      la0 = (R)lam.a[0];
      la1 = (R)lam.a[1];
    }
    // the super-cluster's 64 atoms go to this wave's LDS slice (lane l holds
    // slot l); lane (jl, il) then reads atom c*8 + il for each i-cluster c
    R fix[kScCl], fiy[kScCl], fiz[kScCl];
    wave_sync();
    ipos[lane] = pos[s * kSc + lane];
    ise[lane] = se[s * kSc + lane];
    wave_sync();
#pragma unroll
    for (int c = 0; c < kScCl; ++c) fix[c] = fiy[c] = fiz[c] = R(0);
    const double ox0 = as_const(d.sc_origin)[3 * s], oy0 = as_const(d.sc_origin)[3 * s + 1],
                 oz0 = as_const(d.sc_origin)[3 * s + 2];
    double acc_solv = 0, acc_solu = 0, acc_a0 = 0, acc_a1 = 0, acc_a2 = 0;
    int npair = 0;
    // software pipeline: entry words two ahead, j-cluster data one ahead
    const cptr<int> ejc = as_const(d.ent_jc);
    const cptr<uint32_t> einfo = as_const(d.ent_info);
    const cptr<double> sorg = as_const(d.sc_origin);
    int jc_a = ejc[U.y];
    uint32_t info_a = einfo[U.y];
    int jc_b = jc_a;
    uint32_t info_b = info_a;
    if (U.y + 1 < U.z) {
      jc_b = ejc[U.y + 1];
      info_b = einfo[U.y + 1];
    }
    P4 pj_a = pos[jc_a * kCl + jl];
    P2 qj_a = se[jc_a * kCl + jl];
    const cptr<unsigned long long> emask = as_const(d.ent_mask);
    unsigned long long m_a[kScCl];
#pragma unroll
    for (int c = 0; c < kScCl; ++c) m_a[c] = emask[(size_t)U.y * kScCl + c];
    for (int e = U.y; e < U.z; ++e) {
      unsigned long long mcur[kScCl];
#pragma unroll
      for (int c = 0; c < kScCl; ++c) mcur[c] = m_a[c];
      if (e + 1 < U.z) {
#pragma unroll
        for (int c = 0; c < kScCl; ++c) m_a[c] = emask[(size_t)(e + 1) * kScCl + c];
      }
      const int jc = jc_a;
      const uint32_t info = info_a;
      const P4 pj = pj_a;
      const P2 qj = qj_a;
      jc_a = jc_b;
      info_a = info_b;
      if (e + 1 < U.z) {
        pj_a = pos[jc_a * kCl + jl];
        qj_a = se[jc_a * kCl + jl];
      }
      if (e + 2 < U.z) {
        jc_b = ejc[e + 2];
        info_b = einfo[e + 2];
      }
      const uint32_t imask = info & 0xffu;
      const int kind = (int)((info >> 8) & 3u);
      const int jsl = jc * kCl + jl;
      R fjx = R(0), fjy = R(0), fjz = R(0), eent = R(0);
      // offset of the j-cluster's image from the i-super-cluster origin
      const int code = (int)((info >> 16) & 31u);
      const int sj = jc >> 3;
      const double odx = sorg[3 * sj] + (double)(code % 3 - 1) * L0 - ox0;
      const double ody = sorg[3 * sj + 1] + (double)((code / 3) % 3 - 1) * L1 - oy0;
      const double odz = sorg[3 * sj + 2] + (double)(code / 9 - 1) * L2 - oz0;
      if (kind != KIND_ALCH) {
        const R xj = pj.x + (R)odx, yj = pj.y + (R)ody, zj = pj.z + (R)odz;
#pragma unroll
        for (int c = 0; c < kScCl; ++c) {
          if (!(imask & (1u << c))) continue;
          const bool valid = (mcur[c] >> lane) & 1ull;
          const P4 pi = ipos[c * kCl + il];
          const P2 qi = ise[c * kCl + il];
          const R dx = xj - pi.x, dy = yj - pi.y, dz = zj - pi.z;
          const R r2 = dx * dx + dy * dy + dz * dz;
          const bool inr = valid && r2 < P.rc2;
          npair += __popcll(__ballot(inr));
          PairCore<R, SW> pc;
          pc.eval(r2, inr, qi.x + qj.x, qi.y * qj.y, pi.w * pj.w, P);
          const R u = pc.lj0 * pc.S + pc.el;
          const R fr = pc.flj0 * pc.S - pc.lj0 * pc.rdS + pc.fel;
          const R fs = inr ? fr * pc.rinv2 : R(0);
          eent += inr ? u : R(0);
          const R fx = fs * dx, fy = fs * dy, fz = fs * dz;
          fjx += fx;
          fjy += fy;
          fjz += fz;
          fix[c] -= fx;
          fiy[c] -= fy;
          fiz[c] -= fz;
        }
      } else {
        // FP64 local coordinates from the input positions, in this entry's image
        const int aj = max(0, d.slot_atom[jsl]);
        const double xj = local_coord(d, xin, aj, sj, 0, L0) + odx;
        const double yj = local_coord(d, xin, aj, sj, 1, L1) + ody;
        const double zj = local_coord(d, xin, aj, sj, 2, L2) + odz;
        const int tj = d.atom_type[aj];
#pragma unroll
        for (int c = 0; c < kScCl; ++c) {
          if (!(imask & (1u << c))) continue;
          const bool valid = (mcur[c] >> lane) & 1ull;
          const int ai = max(0, d.slot_atom[s * kSc + c * kCl + il]);
          const double xl = local_coord(d, xin, ai, s, 0, L0), yl = local_coord(d, xin, ai, s, 1, L1),
                       zl = local_coord(d, xin, ai, s, 2, L2);
          const R dx = (R)(xj - xl), dy = (R)(yj - yl), dz = (R)(zj - zl);
          const P4 tp = tpair[d.atom_type[ai] * T + tj];
          R u, fr, rinv2;
          bool inr;
          alch_pair<R, SCHED, SW>(dx, dy, dz, valid, tp, la0, la1, P, u, fr, rinv2, inr, acc_a0, acc_a1, acc_a2);
          npair += __popcll(__ballot(inr));
          const R fs = inr ? fr * rinv2 : R(0);
          const R fx = fs * dx, fy = fs * dy, fz = fs * dz;
          fjx += fx;
          fjy += fy;
          fjz += fz;
          fix[c] -= fx;
          fiy[c] -= fy;
          fiz[c] -= fz;
        }
      }
      fjx = red8(fjx);
      fjy = red8(fjy);
      fjz = red8(fjz);
      if (il == 0) {
        add_fixed(d.ffix + jsl, fjx, fscale, d.flags);
        add_fixed(d.ffix + slots + jsl, fjy, fscale, d.flags);
        add_fixed(d.ffix + 2 * slots + jsl, fjz, fscale, d.flags);
      }
      if (kind == KIND_SOLV) acc_solv += (double)eent;
      else if (kind == KIND_SOLU) acc_solu += (double)eent;
    }
#pragma unroll
    for (int c = 0; c < kScCl; ++c) {
      const R fx = red_jl(fix[c]), fy = red_jl(fiy[c]), fz = red_jl(fiz[c]);
      if (jl == 0) {
        const int sl = s * kSc + c * kCl + il;
        add_fixed(d.ffix + sl, fx, fscale, d.flags);
        add_fixed(d.ffix + slots + sl, fy, fscale, d.flags);
        add_fixed(d.ffix + 2 * slots + sl, fz, fscale, d.flags);
      }
    }
    acc_solv = wave_sum(acc_solv);
    acc_solu = wave_sum(acc_solu);
    acc_a0 = wave_sum(acc_a0);
    acc_a1 = wave_sum(acc_a1);
    acc_a2 = wave_sum(acc_a2);
    if (lane == 0) {
      double* o = d.unit_acc + (size_t)u * NACC;
      o[ACC_SOLV] = acc_solv;
      o[ACC_SOLU] = acc_solu;
      o[ACC_A0] = acc_a0;
      o[ACC_A1] = acc_a1;
      o[ACC_A2] = acc_a2;
      o[ACC_NPAIR] = (double)npair;
    }
  }
}

hipError_t launch_tile(const Dev& d, hipStream_t st, const PotConsts& pc, int precision, int schedule,
                       const TileShape& sh, const double* xin) {
  const dim3 G(sh.blocks), B(kBlk);
  const bool sw = pc.inv_w > 0;
  const double fs = fixed_scale(precision);
  if (precision == 0) {
    const Pot<float> P = make_pot<float>(pc);
    if (schedule == 0) {
      if (sw) hipLaunchKernelGGL((k_tile<float, 0, true>), G, B, 0, st, d, P, sh.xcd, fs, xin);
      else hipLaunchKernelGGL((k_tile<float, 0, false>), G, B, 0, st, d, P, sh.xcd, fs, xin);
    } else {
      if (sw) hipLaunchKernelGGL((k_tile<float, 1, true>), G, B, 0, st, d, P, sh.xcd, fs, xin);
      else hipLaunchKernelGGL((k_tile<float, 1, false>), G, B, 0, st, d, P, sh.xcd, fs, xin);
    }
  } else {
    const Pot<double> P = make_pot<double>(pc);
    if (schedule == 0) {
      if (sw) hipLaunchKernelGGL((k_tile<double, 0, true>), G, B, 0, st, d, P, sh.xcd, fs, xin);
      else hipLaunchKernelGGL((k_tile<double, 0, false>), G, B, 0, st, d, P, sh.xcd, fs, xin);
    } else {
      if (sw) hipLaunchKernelGGL((k_tile<double, 1, true>), G, B, 0, st, d, P, sh.xcd, fs, xin);
      else hipLaunchKernelGGL((k_tile<double, 1, false>), G, B, 0, st, d, P, sh.xcd, fs, xin);
    }
  }
  return hipGetLastError();
}

// ------------------------------------------------------------ per-call helpers

__global__ void k_init(Dev d) {
  if (gtid() == 0) {
    *d.rebuild = 1;
    *d.flags = 0u;
    for (int k = 0; k < 16; ++k) d.ctr[k] = 0;
  }
}

hipError_t launch_init(const Dev& d, hipStream_t st) {
  hipLaunchKernelGGL(k_init, dim3(1), dim3(64), 0, st, d);
  return hipGetLastError();
}

// lambda factors per box; displacement/finite checks; rebuild decision.
// mode: 0 = no rebuild (report skin violations), 1 = automatic, 2 = forced.
__global__ void __launch_bounds__(kBlk) k_prepare(Dev d, const double* __restrict__ pos,
                                                  const double* __restrict__ lambda, int mode, double half_skin2,
                                                  int schedule) {
  const int t = gtid();
  if (t < d.n_reps) {
    double l = lambda ? lambda[t] : 1.0;
    if (!(l >= 0.0 && l <= 1.0)) {
      atomicOr(d.flags, 8u);
      l = l < 0.0 ? 0.0 : (l > 1.0 ? 1.0 : (l == l ? l : 0.0));
    }
    LamState s;
    if (schedule == 0) {
      s.a[0] = fmin(1.0, 2.0 * l);
      s.a[1] = fmax(0.0, 2.0 * l - 1.0);
      s.a[2] = l <= 0.5 ? 2.0 : 0.0;
      s.a[3] = l > 0.5 ? 2.0 : 0.0;
    } else {
      // hA = S32((l - 0.35)/0.65), hB = S22(l) - hA (the paper's eqs. 7-10)
      const double x = (l - 0.35) / 0.65;
      double hA = 0.0, dhA = 0.0;
      if (x > 0.0) {
        const double xc = fmin(x, 1.0);
        hA = xc * xc * xc * xc * (15.0 + xc * (-24.0 + 10.0 * xc));
        dhA = x < 1.0 ? 60.0 * xc * xc * xc * (1.0 - xc) * (1.0 - xc) / 0.65 : 0.0;
      }
      const double s22 = l * l * l * (10.0 + l * (-15.0 + 6.0 * l));
      const double ds22 = 30.0 * l * l * (1.0 - l) * (1.0 - l);
      s.a[0] = hA;
      s.a[1] = s22 - hA;
      s.a[2] = dhA;
      s.a[3] = ds22 - dhA;
    }
    for (int k = 0; k < 4; ++k) s.f[k] = (float)s.a[k];
    d.lam[t] = s;
  }
  if (t == 0) {
    if (mode == 2) __atomic_store_n(d.rebuild, 1, __ATOMIC_RELAXED);
    // arrival counters of the list build's grid barrier (clean after any timeout)
    d.barrier[0] = 0u;
    for (int g = 1; g <= kBarGroups; ++g) d.barrier[kBarStride * g] = 0u;
  }
  const bool have_list = d.ctr[CTR_NBUILD] > 0;
  bool moved = false, bad = false;
  for (int a = t; a < d.n_atoms; a += gthreads()) {
    const double x = pos[3 * a], y = pos[3 * a + 1], z = pos[3 * a + 2];
    if (!(isfinite(x) && isfinite(y) && isfinite(z))) {
      bad = true;
      continue;
    }
    if (!have_list || mode == 2) continue;
    const ReplicaInfo& rp = d.reps[d.grids[d.atom_grid[a]].replica];
    double dd[3] = {x - d.x_build[3 * a], y - d.x_build[3 * a + 1], z - d.x_build[3 * a + 2]};
    double r2 = 0;
    for (int k = 0; k < 3; ++k) {
      dd[k] -= rp.box[k] * rint(dd[k] / rp.box[k]);
      r2 += dd[k] * dd[k];
    }
    if (r2 > half_skin2) moved = true;
  }
  if (bad) atomicOr(d.flags, 4u);
  if (moved) {
    if (mode == 1) __atomic_store_n(d.rebuild, 1, __ATOMIC_RELAXED);
    else atomicOr(d.flags, 2u);
  }
}

hipError_t launch_prepare(const Dev& d, hipStream_t st, const double* pos, const double* lambda, int mode,
                          double half_skin, int schedule) {
  const int g = max(1, min(1024, (max(d.n_atoms, d.n_reps) + kBlk - 1) / kBlk));
  hipLaunchKernelGGL(k_prepare, dim3(g), dim3(kBlk), 0, st, d, pos, lambda, mode, half_skin * half_skin, schedule);
  return hipGetLastError();
}

// Super-cluster-local coordinates (minimum image about the SC origin), the
// charge in the w component, and zeroed force accumulators.
template <typename R>
__global__ void __launch_bounds__(kBlk) k_canon(Dev d, const double* __restrict__ pos) {
  using P4 = typename C4<R>::P4;
  P4* out = reinterpret_cast<P4*>(sizeof(R) == 4 ? (void*)d.pos32 : (void*)d.pos64);
  const int slots = d.sc_cap * kSc;
  for (int sl = gtid(); sl < slots; sl += gthreads()) {
    const int s = sl / kSc;
    if (d.sc_n[s] == 0) continue;
    d.ffix[sl] = 0ull;
    d.ffix[slots + sl] = 0ull;
    d.ffix[2 * slots + sl] = 0ull;
    const int a = d.slot_atom[sl];
    P4 v;
    if (a < 0) {
      v.x = v.y = v.z = v.w = R(0);
    } else {
      const ReplicaInfo& rp = d.reps[d.grids[d.atom_grid[a]].replica];
      double q[3];
      for (int k = 0; k < 3; ++k) q[k] = local_coord(d, pos, a, s, k, rp.box[k]);
      v.x = (R)q[0];
      v.y = (R)q[1];
      v.z = (R)q[2];
      v.w = sizeof(R) == 4 ? (R)d.q32[sl] : (R)d.q64[sl];
    }
    out[sl] = v;
  }
}

hipError_t launch_canon(const Dev& d, hipStream_t st, const double* pos, int precision) {
  const int slots = d.sc_cap * kSc;
  const int g = max(1, min(4096, (slots + kBlk - 1) / kBlk));
  if (precision == 0) hipLaunchKernelGGL(k_canon<float>, dim3(g), dim3(kBlk), 0, st, d, pos);
  else hipLaunchKernelGGL(k_canon<double>, dim3(g), dim3(kBlk), 0, st, d, pos);
  return hipGetLastError();
}

// Blocks [0, K): ordered reduction of the unit partials of box k and the
// energy terms.  Blocks >= K: fixed-point forces -> float64 in atom order.
__global__ void __launch_bounds__(kBlk) k_finalize(Dev d, int schedule, double inv_scale, double* __restrict__ terms,
                                                   double* __restrict__ forces, double* __restrict__ dudl,
                                                   long long* __restrict__ n_pairs) {
  __shared__ double red[NACC][kBlk];
  const int K = d.n_reps;
  if ((int)blockIdx.x < K) {
    const int k = blockIdx.x;
    const int u0 = d.rep_ustart[k], u1 = d.rep_ustart[k + 1];
    double s[NACC] = {0, 0, 0, 0, 0, 0};
    for (int u = u0 + threadIdx.x; u < u1; u += blockDim.x)
      for (int j = 0; j < NACC; ++j) s[j] += d.unit_acc[(size_t)u * NACC + j];
    for (int j = 0; j < NACC; ++j) red[j][threadIdx.x] = s[j];
    __syncthreads();
    for (int off = kBlk / 2; off > 0; off >>= 1) {
      if ((int)threadIdx.x < off)
        for (int j = 0; j < NACC; ++j) red[j][threadIdx.x] += red[j][threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      const double solv = red[ACC_SOLV][0], solu = red[ACC_SOLU][0];
      const double a0 = red[ACC_A0][0], a1 = red[ACC_A1][0], a2 = red[ACC_A2][0];
      const LamState L = d.lam[k];
      double t[kNTerms];
      if (schedule == 0) {
        // a0 = sum lv core S, a1 = sum qq D, a2 = sum d(lv core S)/dlv
        t[0] = solv; t[1] = solu; t[2] = a0; t[3] = L.a[1] * a1; t[4] = 0.0; t[5] = 0.0;
        t[6] = L.a[2] * a2; t[7] = L.a[3] * a1;
      } else {
        // a0 = sum LJ S, a1 = sum qq D, a2 = sum eps u_cap S
        t[0] = solv; t[1] = solu; t[2] = L.a[0] * a0 + L.a[1] * a2; t[3] = L.a[0] * a1;
        t[4] = a0 + a1; t[5] = a2; t[6] = L.a[2] * a0 + L.a[3] * a2; t[7] = L.a[2] * a1;
      }
      t[8] = ((t[0] + t[1]) + t[2]) + t[3];
      t[9] = t[6] + t[7];
      if (terms)
        for (int j = 0; j < kNTerms; ++j) terms[k * kNTerms + j] = t[j];
      if (dudl) dudl[k] = t[9];
      d.last_dudl[k] = t[9];
      if (n_pairs) n_pairs[k] = (long long)red[ACC_NPAIR][0];
    }
    return;
  }
  if (!forces) return;
  const int slots = d.sc_cap * kSc;
  for (int a = (blockIdx.x - K) * blockDim.x + threadIdx.x; a < d.n_atoms; a += (gridDim.x - K) * blockDim.x) {
    const int sl = d.atom_slot[a];
    for (int c = 0; c < 3; ++c) forces[3 * a + c] = (double)(long long)d.ffix[c * slots + sl] * inv_scale;
  }
}

hipError_t launch_finalize(const Dev& d, hipStream_t st, int precision, int schedule, double* terms, double* forces,
                           double* dudl, long long* n_pairs) {
  const int gf = forces ? max(1, min(1024, (d.n_atoms + kBlk - 1) / kBlk)) : 0;
  hipLaunchKernelGGL(k_finalize, dim3(d.n_reps + gf), dim3(kBlk), 0, st, d, schedule, 1.0 / fixed_scale(precision),
                     terms, forces, dudl, n_pairs);
  return hipGetLastError();
}

}  // namespace anb
