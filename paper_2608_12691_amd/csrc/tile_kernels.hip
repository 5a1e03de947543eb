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
//   with DPP lane moves and parked in LDS; i-forces stay in registers.  At
//   the end of the unit both leave as 64-bit fixed-point atomics with one
//   atom per lane (three 64-lane atomics each), so the entry loop issues no
//   memory writes and never waits for one.
// Pair arithmetic is FP32 (or FP64 in the reference path); positions are
// super-cluster-local so that FP32 keeps ~1e-7 A resolution in any box.
// The units of solute super-clusters (every solute-solute and
// solute-solvent entry, about 0.5-3% of the pairs) are evaluated first, in
// FP64 in both kernels (solute_unit): dU/dlambda and the solute terms are
// sums over these pairs alone, with cancellation between them.
#include <hip/hip_runtime.h>

#include <cstring>

#include "anb_internal.h"
#include "anb_kernels.h"
#include "erfc_coeffs.h"
#include "lane_ops.h"
#include "pair_math.h"

namespace anb {

constexpr int kBlk = 256;

// every kernel here runs kBlk-thread blocks (k_init: one block, thread 0
// only); the constant spares the load of the block size at kernel start
__device__ inline int gtid() { return blockIdx.x * kBlk + threadIdx.x; }
__device__ inline int gthreads() { return gridDim.x * kBlk; }

// ------------------------------------------------------------ math by type

__device__ inline float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ inline double rsq(double x) { return 1.0 / sqrt(x); }
__device__ inline float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double rcp(double x) { return 1.0 / x; }
__device__ inline float clamp01(float x) { return __builtin_amdgcn_fmed3f(x, 0.0f, 1.0f); }
__device__ inline double clamp01(double x) { return fmin(fmax(x, 0.0), 1.0); }

__constant__ double kErfc64ChebDev[ANB_ERFC64_DEG + 1] = {
#define X(i) kErfc64Cheb[i]
  X(0), X(1), X(2), X(3), X(4), X(5), X(6), X(7), X(8), X(9), X(10), X(11), X(12), X(13), X(14), X(15), X(16)
#undef X
};
// FP64 erfc(x) and exp(-x^2) for 0 <= x <= ANB_ERFC_XMAX from the Chebyshev
// series of erfc_coeffs.h (relative error ~1e-15): a few registers, where
// the library erfc needs many (used in the FP32 kernel's FP64 pass)
__device__ inline void erfc_exp_cheb(double x, double& ec, double& ex) {
  const double t = 1.0 / fma(ANB_ERFC64_P, x, 1.0);
  const double s = (2.0 * t - (ANB_ERFC64_A + 1.0)) / (1.0 - ANB_ERFC64_A);
  const double s2 = 2.0 * s;
  double b1 = 0.0, b2 = 0.0;
#pragma unroll 1
  for (int k = ANB_ERFC64_DEG; k >= 1; --k) {
    const double b0 = fma(s2, b1, kErfc64ChebDev[k] - b2);
    b2 = b1;
    b1 = b0;
  }
  ex = exp(-x * x);
  ec = t * ex * fma(s, b1, kErfc64ChebDev[0] - b2);
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
  R rc2, rc, rs, inv_w, alpha, A, B, c2a, sca, inv_h, rs2;
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
  o.inv_h = (R)p.inv_h;
  o.rs2 = p.inv_w > 0 ? (R)(p.rs * p.rs) : (R)p.rc2;
  return o;
}

// Switched LJ, DSF and the scalar pair force.  Lanes outside the cutoff or
// masked out get r2 := 1 so every value stays finite (callers select their
// outputs to zero or run the lanes of in-range pairs only).  The
// electrostatic factors by route E: kErfcTable, the FP32 cubic pieces in tab
// (LDS) of r D(r) and of r times -r dD/dr, smooth functions of r whose
// shifts were formed in FP64 (FP64 takes the library functions);
// kErfcFit, erfc and the Gaussian term from the FP32 rational fit (FP64:
// the library); kErfcCheb, the FP64 Chebyshev series (few registers; FP32
// takes the rational fit).
enum { kErfcFit = 0, kErfcTable = 1, kErfcCheb = 2 };

template <typename R, bool SW>
struct PairCore {
  R r2s, rinv, rinv2, r;
  R lj0, flj0;   // unswitched LJ and -r dLJ/dr
  R S, rdS;      // switch and r dS/dr
  R el, fel;     // q q D(r) and -r d(q q D)/dr
  template <int E>
  __device__ inline void eval(R r2, bool inr, R sij, R e4, R qq, const Pot<R>& P, const float4* tab) {
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
    R ec, gx;
    if constexpr (sizeof(R) == 4 && E == kErfcTable) {
      const float u = r * P.inv_h;  // exact; 0 <= u <= kDsfN for r <= rc
      const float4 fa = tab[2 * (int)u], fb = tab[2 * (int)u + 1];
      const float t = __builtin_amdgcn_fractf(u);
      // r D(r) and r (-r dD/dr), then one factor q q / r for both
      const float rd = fmaf(fmaf(fmaf(fa.w, t, fa.z), t, fa.y), t, fa.x);
      const float rf = fmaf(fmaf(fmaf(fb.w, t, fb.z), t, fb.y), t, fb.x);
      const float qr = qq * rinv;
      el = qr * rd;
      fel = qr * rf;
      return;
    } else if constexpr (sizeof(R) == 8 && E == kErfcCheb) {
      R ex;
      erfc_exp_cheb(P.alpha * r, ec, ex);
      gx = P.c2a * ex;
    } else {
      R ex;
      erfc_exp(P.alpha * r, ec, ex);
      gx = P.c2a * ex;
    }
    const R erinv = ec * rinv;
    el = qq * (erinv - P.A + P.B * (r - P.rc));
    fel = qq * (erinv + gx - P.B * r);
  }
};

// ------------------------------------------------------------ wave sums

// Sum over the wave, the same value in every lane: within rows of 16 by DPP
// lane moves (pairs, quads, mirrored halves, mirrored rows), then across
// rows with the lane-swap instructions; each step adds two equal partial
// sums, so every lane ends with the same bits.
template <int kCtrl>
__device__ inline double dpp64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), kCtrl, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), kCtrl, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ inline double wave_sum(double v) {
  v += dpp64<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp64<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp64<0x141>(v);  // row_half_mirror
  v += dpp64<0x140>(v);  // row_mirror
  double a = v, b = v;
  swap16(a, b);
  v = a + b;
  a = v;
  b = v;
  swap32(a, b);
  return a + b;
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


// Fixed-point add of one value per active lane with no per-lane branch
// around the atomic; out-of-range or NaN values add zero and raise the
// overflow flag.
// Below 2^51 the integer nearest to x is read from the bits of
// x + 1.5 * 2^52 (round to nearest even, as __double2ll_rn); larger values,
// rare, take the general conversion.
template <typename R>
__device__ inline void add_fixed_lanes(unsigned long long* p, R v, double scale, unsigned int* flags, bool active) {
  const double x = (double)v * scale;
  unsigned long long q;
  if (__builtin_expect(__ballot(active && !(fabs(x) < 2251799813685248.0)) != 0, 0)) {
    const bool ok = fabs(x) < 4.611686018427388e18;  // |f| < 2^62 / scale
    if (__ballot(active && !ok) && (threadIdx.x & 63) == 0) atomicOr(flags, 1u);
    q = ok ? (unsigned long long)__double2ll_rn(x) : 0ull;
  } else {
    q = (unsigned long long)(__double_as_longlong(x + 6755399441055744.0) - 0x4338000000000000ll);
  }
  if (active) atomicAdd(p, q);
}

// ------------------------------------------------------------ tile kernel

// The lambda-dependent terms of a solute-solvent pair from its evaluated
// core: u and -r du/dr (fr), and the pair's contributions to the three
// sums a0..a2 (Beutler: soft-core vdw energy, electrostatic energy,
// dU/dlambda_vdw per unit lambda_v'; LBF: vdw, electrostatic and u_cap
// bases).
template <typename R, int SCHED, bool SW>
__device__ inline void alch_terms(const PairCore<R, SW>& pc, R sij, R e4, R inv_s6, R lv_or_hA, R le_or_hB,
                                  const Pot<R>& P, bool inr, R& u, R& fr, double& a0, double& a1, double& a2) {
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

// A solute-solvent pair evaluated by the unit loop itself (FP64 inputs
// rounded once, the loop's precision, erfc from the rational fit).  The unit
// loop evaluates any unit it is given; solute units are routed to
// solute_unit instead, so this path does not run in the current routing.
// It stays because the loop compiled without it measured slower (the
// compiler then spilled the solvent path's registers).
template <typename R, int SCHED, bool SW>
__device__ inline void alch_pair(R dx, R dy, R dz, bool valid, const typename C4<R>::P4& tp, R lv_or_hA, R le_or_hB,
                                 const Pot<R>& P, const float4* tab, R& u, R& fr, R& rinv2, bool& inr,
                                 double& a0, double& a1, double& a2) {
  const R r2 = dx * dx + dy * dy + dz * dz;
  inr = valid && r2 < P.rc2;
  PairCore<R, SW> pc;
  pc.template eval<kErfcFit>(r2, inr, tp.x, tp.y, tp.z, P, tab);
  rinv2 = pc.rinv2;
  alch_terms<R, SCHED, SW>(pc, tp.x, tp.y, tp.w, lv_or_hA, le_or_hB, P, inr, u, fr, a0, a1, a2);
}

// FP64 constants of the solute units, read from the workspace (scalar loads
// where they are used) rather than passed as kernel arguments, which would
// hold scalar registers through the whole FP32 kernel.
static_assert(sizeof(Pot<double>) == 11 * sizeof(double) && 11 <= kPot64Words, "workspace image of Pot<double>");
void pot64_words(const PotConsts& pc, double* out) {
  const Pot<double> p = make_pot<double>(pc);
  for (int i = 0; i < kPot64Words; ++i) out[i] = 0.0;
  std::memcpy(out, &p, sizeof(p));
}
__device__ inline Pot<double> load_pot64(const double* w) {
  const cptr<double> c = as_const(w);  // wave-uniform: scalar loads
  Pot<double> p;
  p.rc2 = c[0];
  p.rc = c[1];
  p.rs = c[2];
  p.inv_w = c[3];
  p.alpha = c[4];
  p.A = c[5];
  p.B = c[6];
  p.c2a = c[7];
  p.sca = c[8];
  p.inv_h = c[9];
  p.rs2 = c[10];
  return p;
}

// One unit of a solute super-cluster, by the whole wave, in FP64 from FP64
// inputs: its entries are the solute-solute pairs (plain) and the
// solute-solvent pairs (soft core or LBF), the only pairs that dU/dlambda
// and the solute terms sum over.  The super-cluster's 64 slots (FP64
// position, q sqrt(k_e), sigma/2, 2 sqrt(eps)) are staged in the wave's LDS
// slice `si` (six arrays of 64), one load per lane; lane (jl, il) then takes
// j-atom jl of an entry's j-cluster (loaded one entry ahead) and, for each
// i-cluster c of its mask, i-atom il from LDS.  Pair parameters follow the
// combination rule from the per-slot FP64 values.  j-forces are summed over
// the i-clusters and il, i-forces over jl, and both leave as 64-bit
// fixed-point atomics (a few per entry: these units are small).  The unit's
// sums go to its accumulator slots.  kCheb: erfc from the Chebyshev series
// (few registers; the FP32 kernel) or the library (the FP64 kernel).
template <int SCHED, bool SW, bool kCheb>
__device__ inline void solute_unit(const Dev& d, const Pot<double>& P, const float4* dsf, const int4& U, int u,
                                   double fscale, double* const* si) {
  const int lane = threadIdx.x & 63;
  const int il = lane & 7, jl = lane >> 3;
  const int s = U.x;
  const size_t slots = (size_t)d.sc_cap * kSc;
  const LamState lam = d.lam[unit_rep(U.w)];
  const cptr<uint32_t> einfo = as_const(d.ent_info);
  const cptr<unsigned long long> emask = as_const(d.ent_mask);
  // j-data of entry e: position moved into the i-super-cluster's frame, q, sigma/2, 2 sqrt(eps)
  double4 nj = make_double4(0.0, 0.0, 0.0, 0.0);
  double2 nje = make_double2(0.0, 0.0);
  int njsl = 0;
  auto load_j = [&](int e) {
    njsl = d.ent_jc[e] * kCl + jl;
    const double4 off = d.ent_off[e];
    const double4 pj = d.pos64[njsl];
    nje = d.se64[njsl];
    nj = make_double4(pj.x + off.x, pj.y + off.y, pj.z + off.z, pj.w);
  };
  if (U.y < U.z) load_j(U.y);  // in flight while the slots are staged
  {
    const double4 pi = d.pos64[s * kSc + lane];  // .w: q sqrt(k_e)
    const double2 ei = d.se64[s * kSc + lane];   // sigma/2, 2 sqrt(eps)
    wave_sync();
    si[0][lane] = pi.x;
    si[1][lane] = pi.y;
    si[2][lane] = pi.z;
    si[3][lane] = pi.w;
    si[4][lane] = ei.x;
    si[5][lane] = ei.y;
    wave_sync();
  }
  double e_solu = 0.0, a0 = 0.0, a1 = 0.0, a2 = 0.0;
  int npair = 0;
  for (int e = U.y; e < U.z; ++e) {
    const double4 pj = nj;
    const double2 ej = nje;
    const int jsl = njsl;
    if (e + 1 < U.z) load_j(e + 1);
    const uint32_t info = einfo[e];
    const uint32_t imask = info & 0xffu;
    const bool alch = ((info >> 8) & 3u) == (uint32_t)KIND_ALCH;
    double fjx = 0.0, fjy = 0.0, fjz = 0.0;
#pragma unroll 1
    for (int c = 0; c < kScCl; ++c) {
      if (!(imask & (1u << c))) continue;
      const int src = c * kCl + il;
      const double dx = pj.x - si[0][src], dy = pj.y - si[1][src], dz = pj.z - si[2][src];
      const double sij = si[4][src] + ej.x;
      // padding slots carry sigma 0 (their lanes are masked out)
      const double s2 = sij > 0.0 ? sij * sij : 1.0;
      const double4 tp = make_double4(sij, si[5][src] * ej.y, si[3][src] * pj.w, 1.0 / (s2 * s2 * s2));
      const bool valid = __builtin_amdgcn_inverse_ballot_w64(emask[(size_t)e * kScCl + c]);
      const double r2 = dx * dx + dy * dy + dz * dz;
      const bool inr = valid && r2 < P.rc2;
      PairCore<double, SW> pc;
      pc.template eval<kCheb ? kErfcCheb : kErfcFit>(r2, inr, tp.x, tp.y, tp.z, P, dsf);
      double uu, fr;
      if (alch) {
        alch_terms<double, SCHED, SW>(pc, tp.x, tp.y, tp.w, lam.a[0], lam.a[1], P, inr, uu, fr, a0, a1, a2);
      } else {
        uu = pc.lj0 * pc.S + pc.el;
        fr = pc.flj0 * pc.S - pc.lj0 * pc.rdS + pc.fel;
        if (inr) e_solu += uu;
      }
      npair += __popcll(__ballot(inr));
      const double fs = inr ? fr * pc.rinv2 : 0.0;
      const double fx = fs * dx, fy = fs * dy, fz = fs * dz;
      fjx += fx;
      fjy += fy;
      fjz += fz;
      const double gx = red_jl(fx), gy = red_jl(fy), gz = red_jl(fz);
      const int isl = s * kSc + src;
      add_fixed_lanes(d.ffix + isl, -gx, fscale, d.flags, jl == 0);
      add_fixed_lanes(d.ffix + slots + isl, -gy, fscale, d.flags, jl == 0);
      add_fixed_lanes(d.ffix + 2 * slots + isl, -gz, fscale, d.flags, jl == 0);
    }
    fjx = red8(fjx);
    fjy = red8(fjy);
    fjz = red8(fjz);
    add_fixed_lanes(d.ffix + jsl, fjx, fscale, d.flags, il == 0);
    add_fixed_lanes(d.ffix + slots + jsl, fjy, fscale, d.flags, il == 0);
    add_fixed_lanes(d.ffix + 2 * slots + jsl, fjz, fscale, d.flags, il == 0);
  }
  e_solu = wave_sum(e_solu);
  a0 = wave_sum(a0);
  a1 = wave_sum(a1);
  a2 = wave_sum(a2);
  if (lane == 0) {
    const size_t UC = (size_t)d.unit_cap;
    double* o = d.unit_acc + u;
    o[ACC_SOLV * UC] = 0.0;
    o[ACC_SOLU * UC] = e_solu;
    o[ACC_A0 * UC] = a0;
    o[ACC_A1 * UC] = a1;
    o[ACC_A2 * UC] = a2;
    o[ACC_NPAIR * UC] = (double)npair;
  }
  wave_sync();  // the LDS slice is the unit loop's next
}

template <typename R, int SCHED, bool SW>
__global__ void __launch_bounds__(kBlk, sizeof(R) == 4 ? 4 : 1) k_tile(Dev d, Pot<R> P, double fscale, const double* __restrict__ xin) {
  using P4 = typename C4<R>::P4;
  using P2 = typename C4<R>::P2;
  const P4* __restrict__ pos = reinterpret_cast<const P4*>(sizeof(R) == 4 ? (const void*)d.pos32 : (const void*)d.pos64);
  const P2* __restrict__ se = reinterpret_cast<const P2*>(sizeof(R) == 4 ? (const void*)d.se32 : (const void*)d.se64);
  const P4* __restrict__ tpair = reinterpret_cast<const P4*>(sizeof(R) == 4 ? (const void*)d.tp32 : (const void*)d.tp64);
  const double4* __restrict__ pos64 = d.pos64;
  const int slots = d.sc_cap * kSc;
  const int T = d.n_types;
  const int lane = threadIdx.x & 63;
  __shared__ P4 ipos_all[kBlk];
  __shared__ P2 ise_all[kBlk];
  // j-forces of up to 8 entries (entry slot k, j-atom jl at k * 8 + jl)
  __shared__ P4 jf_all[kBlk];
  __shared__ int jsl_all[kBlk];
  P4* jf = jf_all + (threadIdx.x & ~63);
  int* jslb = jsl_all + (threadIdx.x & ~63);
  // j-cluster data of the unit's entries (same layout), positions already
  // moved into the i-super-cluster's frame and entry image
  __shared__ P4 jpos_all[kBlk];
  __shared__ P2 jse_all[kBlk];
  P4* jpos = jpos_all + (threadIdx.x & ~63);
  P2* jse = jse_all + (threadIdx.x & ~63);
  // lane-private FP64 sums of the rare entry kinds (solute-solute and
  // solute-solvent) live in LDS, keeping registers for the common path
  __shared__ double rare_all[4][kBlk];
  double* rare0 = &rare_all[0][threadIdx.x];  // solute-solute energy
  double* rare1 = &rare_all[1][threadIdx.x];  // a0 .. a2 of the alchemical pairs
  double* rare2 = &rare_all[2][threadIdx.x];
  double* rare3 = &rare_all[3][threadIdx.x];
  // the solute phase (before the unit loop uses LDS) stages its super-cluster's
  // FP64 slot data in this wave's slices of rare_all and jpos_all
  double* const sol_lds[6] = {&rare_all[0][threadIdx.x & ~63], &rare_all[1][threadIdx.x & ~63],
                              &rare_all[2][threadIdx.x & ~63], &rare_all[3][threadIdx.x & ~63],
                              reinterpret_cast<double*>(jpos_all + (threadIdx.x & ~63)),
                              reinterpret_cast<double*>(jpos_all + (threadIdx.x & ~63)) + 64};
  P4* ipos = ipos_all + (threadIdx.x & ~63);
  P2* ise = ise_all + (threadIdx.x & ~63);
  // i-forces of the solute-solvent entries of the current super-cluster,
  // already summed over jl (slot c * 8 + il of each component)
  __shared__ R fia_all[kBlk / 64][3][kSc];
  R* fia = &fia_all[threadIdx.x >> 6][0][0];
  const int il = lane & 7, jl = lane >> 3;
  // Unit range of this wave: equal runs of units (the unit cuts already cap
  // each unit's tiles; runs keep a super-cluster's units on one wave).  The
  // wave index is made provably uniform: unit and entry indices then live in
  // scalar registers.  The wave's start record (written with the units for
  // this wave count) gives the run and its first unit without waiting on
  // the unit count; for another wave count the run follows from the count.
  // (Asked for before the table below, so that the two loads overlap.)
  const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nw = gridDim.x * (kBlk / 64), w = blockIdx.x * (kBlk / 64) + wib;
  const int4 wrec = d.wrec[w];
  const int4 wu0 = d.wrec_u0[w];
  const int rec_waves = d.ctr[CTR_WAVES], n_units = d.ctr[CTR_NUNIT];
  // FP32 DSF pieces, once per block
  __shared__ float4 dsf[sizeof(R) == 4 ? kDsfEntries : 1];
  if (sizeof(R) == 4) {
    for (int i = threadIdx.x; i < kDsfEntries; i += kBlk) dsf[i] = d.dsf32[i];
    __syncthreads();
  }
  const bool rec = rec_waves == nw;
  int ub, nr;
  if (rec) {
    ub = wrec.x;
    nr = wrec.y;
  } else {
    ub = (int)((long long)n_units * w / nw);
    nr = (int)((long long)n_units * (w + 1) / nw) - ub;
  }
  // i-forces of the current super-cluster, carried over consecutive units
  // of the same super-cluster; they leave when it changes: summed over jl,
  // lane (jl, il) then takes i-cluster c = jl so that lane l holds slot
  // s * 64 + l, and three 64-lane atomics write them
  R fix[kScCl], fiy[kScCl], fiz[kScCl];
  int cur_s = -1;
  // Force atomics wait: the j-forces of a unit and the i-forces of a
  // finished super-cluster are issued after the next unit's loads, so that
  // those loads do not queue behind them (FP32; the FP64 kernel, at its
  // register limit, issues them at once).
  constexpr bool kDefer = sizeof(R) == 4;
  P4 pj;  // pending j-forces (lane l: slot pj_sl of entry l / 8)
  int pj_sl = 0;
  bool pj_have = false;
  R pi_x = R(0), pi_y = R(0), pi_z = R(0);  // pending i-forces of super-cluster pi_s
  int pi_s = -1;
  auto reduce_i = [&]() {
    const bool odd8 = (lane & 8) != 0;
    wave_sync();
    pi_x = scatter_jl(fix, odd8) + fia[lane];
    pi_y = scatter_jl(fiy, odd8) + fia[kSc + lane];
    pi_z = scatter_jl(fiz, odd8) + fia[2 * kSc + lane];
    pi_s = cur_s;
  };
  auto put_pending = [&]() {
    if (pj_have) {
      const bool on = pj_sl >= 0;
      const int sl = on ? pj_sl : 0;
      add_fixed_lanes(d.ffix + sl, pj.x, fscale, d.flags, on);
      add_fixed_lanes(d.ffix + slots + sl, pj.y, fscale, d.flags, on);
      add_fixed_lanes(d.ffix + 2 * slots + sl, pj.z, fscale, d.flags, on);
      pj_have = false;
    }
    if (pi_s >= 0) {
      const int sl = pi_s * kSc + lane;
      add_fixed_lanes(d.ffix + sl, pi_x, fscale, d.flags, true);
      add_fixed_lanes(d.ffix + slots + sl, pi_y, fscale, d.flags, true);
      add_fixed_lanes(d.ffix + 2 * slots + sl, pi_z, fscale, d.flags, true);
      pi_s = -1;
    }
  };
  // Unit headers of this wave, lane i holding unit ub + 64 m + i (vector
  // loads, read back with lane reads), and the per-lane entry data of the
  // next unit loaded one unit ahead: lane (k, t) takes entry U.y + k.
  int4 hdr = make_int4(0, 0, 0, 0);
  auto load_hdrs = [&](int base) {
    const int r = base + lane;
    if (r < nr) hdr = d.units[ub + r];
  };
  auto header = [&](int r) {
    const int i = r & 63;
    return make_int4(__builtin_amdgcn_readlane(hdr.x, i), __builtin_amdgcn_readlane(hdr.y, i),
                     __builtin_amdgcn_readlane(hdr.z, i), __builtin_amdgcn_readlane(hdr.w, i));
  };
  // Solute units first, in FP64, before the FP32 state below is live (runs
  // the start record marks as free of them skip this); a wave left with
  // nothing else ends here (the loop below would only load and flush an
  // empty super-cluster)
  if (nr > 0) load_hdrs(0);
  int n_sol = 0;
  const bool scan = !rec || wrec.z != 0;
  if (scan) {
    for (int r = 0; r < nr; ++r) {
      if (r > 0 && (r & 63) == 0) load_hdrs(r);
      const int4 V = header(r);
      if (__builtin_expect((V.w & kUnitSolute) != 0, 0)) {
        const Pot<double> P64 = load_pot64(d.pot64);
        solute_unit<SCHED, SW, sizeof(R) == 4>(d, P64, dsf, V, ub + r, fscale, sol_lds);
        ++n_sol;
      }
    }
  }
  if (n_sol == nr) return;
  int n_jc = 0;
  uint32_t n_inf = 0;
  double4 n_off = make_double4(0.0, 0.0, 0.0, 0.0);
  auto load_entries = [&](const int4& V) {
    const int e = V.y + (lane >> 3);
    n_jc = 0;
    n_inf = 0;
    n_off = make_double4(0.0, 0.0, 0.0, 0.0);
    if (e < V.z) {
      n_jc = d.ent_jc[e];
      n_inf = d.ent_info[e];
      n_off = d.ent_off[e];
    }
  };
  bool have_next = false;
  if (nr > 0) {
    if (nr > 64 && scan) load_hdrs(0);  // the solute pass moved on
    if (rec) {
      // the first unit's entry data from the start record
      const int k = lane >> 3;
      n_jc = d.wrec_jc[w * kMaxEpu + k];
      n_inf = d.wrec_info[w * kMaxEpu + k];
      n_off = d.wrec_off[w * kMaxEpu + k];
    } else {
      load_entries(header(0));
    }
    have_next = true;
  }
  for (int r = 0; r < nr; ++r) {
    if (r > 0 && (r & 63) == 0) load_hdrs(r);  // past 64 units (large boxes)
    int4 U = r == 0 && rec ? wu0 : header(r);
    const int u = ub + r;
    // a solute unit (done by the FP64 pass above) enters as an empty unit of
    // the current super-cluster: no entries, no change of super-cluster, no
    // accumulator write (skipping it with a second loop edge instead made
    // the compiler spill this loop's registers)
    const bool sol = (U.w & kUnitSolute) != 0;
    if (sol) {
      U.x = cur_s < 0 ? U.x : cur_s;
      U.z = U.y;
    }
    if (!have_next) load_entries(U);
    const int c_jc = n_jc;
    const uint32_t c_inf = n_inf;
    const double4 c_off = n_off;
    // the next unit's entry data is asked for once this unit's j-data is
    have_next = r + 1 < nr && ((r + 1) & 63) != 0;
    const int s = U.x;
    const LamState lam = d.lam[unit_rep(U.w)];
    R la0, la1;
    if (sizeof(R) == 4) {
      la0 = (R)lam.f[0];
      la1 = (R)lam.f[1];
    } else {
      la0 = (R)lam.a[0];
      la1 = (R)lam.a[1];
    }
    const bool new_s = s != cur_s;
    P4 ip;
    P2 iq;
    if (new_s) {
      if (cur_s >= 0) {
        reduce_i();
        if (!kDefer) put_pending();
      }
      // the super-cluster's 64 atoms (lane l: slot l)
      ip = pos[s * kSc + lane];
      iq = se[s * kSc + lane];
      if (!kDefer) {
        // straight to LDS: the FP64 kernel holds no extra registers here
        wave_sync();
        ipos[lane] = ip;
        ise[lane] = iq;
        fia[lane] = fia[kSc + lane] = fia[2 * kSc + lane] = R(0);
#pragma unroll
        for (int c = 0; c < kScCl; ++c) fix[c] = fiy[c] = fiz[c] = R(0);
        cur_s = s;
        wave_sync();
      }
    }
    double acc_solv = 0;
    bool rare = false;  // wave-uniform: the unit had a solute-solute or solute-solvent entry
    *rare0 = *rare1 = *rare2 = *rare3 = 0.0;
    int npair = 0;
    unsigned long long alch_bits;
    // j-cluster data of all entries of the unit, one load per lane: lane
    // (k, t) takes atom t of entry U.y + k (units hold at most 8 entries)
    {
      const int k = lane >> 3, t = lane & 7, e = U.y + k;
      P4 v;
      P2 q;
      v.x = v.y = v.z = v.w = R(0);
      q.x = q.y = R(0);
      int jsl = 0;
      const uint32_t inf = c_inf;
      if (e < U.z) {
        jsl = c_jc * kCl + t;
        v = pos[jsl];
        q = se[jsl];
      }
      if (have_next) load_entries(header(r + 1));
      put_pending();
      // offset of the j-cluster's image from the i-super-cluster origin
      v.x += (R)c_off.x;
      v.y += (R)c_off.y;
      v.z += (R)c_off.z;
      wave_sync();
      if (kDefer && new_s) {
        // lane (jl, il) then reads atom c*8 + il of i-cluster c
        ipos[lane] = ip;
        ise[lane] = iq;
        fia[lane] = fia[kSc + lane] = fia[2 * kSc + lane] = R(0);
#pragma unroll
        for (int c = 0; c < kScCl; ++c) fix[c] = fiy[c] = fiz[c] = R(0);
        cur_s = s;
      }
      jpos[lane] = v;
      jse[lane] = q;
      jslb[lane] = jsl;
      wave_sync();
      // one bit per solute-solvent entry (bit 8 k)
      alch_bits = __ballot(e < U.z && t == 0 && ((inf >> 8) & 3u) == (uint32_t)KIND_ALCH);
    }
    const cptr<uint32_t> einfo = as_const(d.ent_info);
    const cptr<unsigned long long> emask = as_const(d.ent_mask);
    // Plain entries (solvent-solvent and solute-solute); entry words and
    // pair masks are read one entry ahead (scalar loads).
    uint32_t info_a = einfo[U.y];
    unsigned long long m_a[kScCl];
#pragma unroll
    for (int c = 0; c < kScCl; ++c) m_a[c] = emask[(size_t)U.y * kScCl + c];
    for (int e = U.y; e < U.z; ++e) {
      const int k = e - U.y;  // entry slot in this unit
      unsigned long long mcur[kScCl];
#pragma unroll
      for (int c = 0; c < kScCl; ++c) mcur[c] = m_a[c];
      const uint32_t info = info_a;
      if (e + 1 < U.z) {
        info_a = einfo[e + 1];
#pragma unroll
        for (int c = 0; c < kScCl; ++c) m_a[c] = emask[(size_t)(e + 1) * kScCl + c];
      }
      if (((info >> 8) & 3u) == (uint32_t)KIND_ALCH) continue;  // second pass
      const uint32_t imask = info & 0xffu;
      R fjx = R(0), fjy = R(0), fjz = R(0), eent = R(0);
      const P4 pj = jpos[k * kCl + jl];
      const P2 qj = jse[k * kCl + jl];
      const R xj = pj.x, yj = pj.y, zj = pj.z;
      // i-cluster data one cluster ahead (LDS reads are always in bounds)
      P4 pin = ipos[il];
      P2 qin = ise[il];
#pragma unroll
      for (int c = 0; c < kScCl; ++c) {
        const P4 pi = pin;
        const P2 qi = qin;
        if (c + 1 < kScCl) {
          pin = ipos[(c + 1) * kCl + il];
          qin = ise[(c + 1) * kCl + il];
        }
        if (!(imask & (1u << c))) continue;
        const R dx = xj - pi.x, dy = yj - pi.y, dz = zj - pi.z;
        const R r2 = dx * dx + dy * dy + dz * dz;
        // the pair mask is a lane mask: combine it on the scalar unit
        const unsigned long long inm = __ballot(r2 < P.rc2) & mcur[c];
        if (inm == 0) continue;  // the whole 64-pair tile has moved out of range
        npair += __popcll(inm);
        // only the lanes of in-range pairs execute the pair math
        // FP32 tiles with no in-range pair in the switching shell skip the
        // switch (in the FP64 kernel the second copy of the pair math costs
        // more than it saves)
        const bool shell = SW && (sizeof(R) == 8 || (__ballot(r2 > P.rs2) & inm) != 0);
        if (__builtin_amdgcn_inverse_ballot_w64(inm)) {
          R u, fr, rinv2;
          if (shell) {
            PairCore<R, true> pc;
            pc.template eval<kErfcTable>(r2, true, qi.x + qj.x, qi.y * qj.y, pi.w * pj.w, P, dsf);
            u = pc.lj0 * pc.S + pc.el;
            fr = pc.flj0 * pc.S - pc.lj0 * pc.rdS + pc.fel;
            rinv2 = pc.rinv2;
          } else {
            PairCore<R, false> pc;
            pc.template eval<kErfcTable>(r2, true, qi.x + qj.x, qi.y * qj.y, pi.w * pj.w, P, dsf);
            u = pc.lj0 + pc.el;
            fr = pc.flj0 + pc.fel;
            rinv2 = pc.rinv2;
          }
          const R fs = fr * rinv2;
          eent += u;
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
        P4 v;
        v.x = fjx;
        v.y = fjy;
        v.z = fjz;
        v.w = R(0);
        jf[k * kCl + jl] = v;
      }
      if (((info >> 8) & 3u) == (uint32_t)KIND_SOLV) {
        acc_solv += (double)eent;
      } else {
        *rare0 += (double)eent;
        rare = true;
      }
    }
    // Solute-solvent entries (rare): FP64 local coordinates (written by the
    // canon pass for every slot) moved into the entry's image and rounded
    // once per displacement; i-forces summed over jl into LDS.  The register
    // i-forces move to LDS first, so they hold no registers in this pass.
    if (alch_bits) {
      const bool odd8 = (lane & 8) != 0;
      const R gx = scatter_jl(fix, odd8), gy = scatter_jl(fiy, odd8), gz = scatter_jl(fiz, odd8);
      wave_sync();
      fia[lane] += gx;
      fia[kSc + lane] += gy;
      fia[2 * kSc + lane] += gz;
      wave_sync();
#pragma unroll
      for (int c = 0; c < kScCl; ++c) fix[c] = fiy[c] = fiz[c] = R(0);
    }
    for (unsigned long long ab = alch_bits; ab; ab &= ab - 1) {
      const int k = __builtin_ctzll(ab) >> 3;
      const int e = U.y + k;
      const uint32_t info = einfo[e];
      const uint32_t imask = info & 0xffu;
      const int jsl = jslb[k * kCl + jl];
      const double4 off = d.ent_off[e];
      const double4 pj64 = pos64[jsl];
      const double xj = pj64.x + off.x, yj = pj64.y + off.y, zj = pj64.z + off.z;
      const int tj = d.slot_type[jsl];
      R fjx = R(0), fjy = R(0), fjz = R(0);
      double a0 = 0, a1 = 0, a2 = 0;
#pragma unroll 1
      for (int c = 0; c < kScCl; ++c) {
        if (!(imask & (1u << c))) continue;
        const int isl = s * kSc + c * kCl + il;
        const double4 pi64 = pos64[isl];
        const R dx = (R)(xj - pi64.x), dy = (R)(yj - pi64.y), dz = (R)(zj - pi64.z);
        const P4 tp = tpair[d.slot_type[isl] * T + tj];
        R u, fr, rinv2;
        bool inr;
        const bool valid = __builtin_amdgcn_inverse_ballot_w64(emask[(size_t)e * kScCl + c]);
        alch_pair<R, SCHED, SW>(dx, dy, dz, valid, tp, la0, la1, P, dsf, u, fr, rinv2, inr, a0, a1, a2);
        npair += __popcll(__ballot(inr));
        const R fs = inr ? fr * rinv2 : R(0);
        const R fx = fs * dx, fy = fs * dy, fz = fs * dz;
        fjx += fx;
        fjy += fy;
        fjz += fz;
        const R gx = red_jl(fx), gy = red_jl(fy), gz = red_jl(fz);
        if (jl == 0) {
          fia[c * kCl + il] -= gx;
          fia[kSc + c * kCl + il] -= gy;
          fia[2 * kSc + c * kCl + il] -= gz;
        }
      }
      fjx = red8(fjx);
      fjy = red8(fjy);
      fjz = red8(fjz);
      if (il == 0) {
        P4 v;
        v.x = fjx;
        v.y = fjy;
        v.z = fjz;
        v.w = R(0);
        jf[k * kCl + jl] = v;
      }
      *rare1 += a0;
      *rare2 += a1;
      *rare3 += a2;
      rare = true;
    }
    // j-forces parked by the entries of this unit, to registers
    wave_sync();
    {
      const bool have = lane < (U.z - U.y) * kCl;
      pj.x = pj.y = pj.z = pj.w = R(0);
      pj_sl = -1;
      if (have) {
        pj = jf[lane];
        pj_sl = jslb[lane];
      }
      pj_have = true;
      if (!kDefer) put_pending();
    }
    wave_sync();
    acc_solv = wave_sum(acc_solv);
    double acc_solu = 0, acc_a0 = 0, acc_a1 = 0, acc_a2 = 0;
    if (rare) {
      acc_solu = wave_sum(*rare0);
      acc_a0 = wave_sum(*rare1);
      acc_a1 = wave_sum(*rare2);
      acc_a2 = wave_sum(*rare3);
    }
    if (lane == 0 && !sol) {
      const size_t U = (size_t)d.unit_cap;
      double* o = d.unit_acc + u;
      o[ACC_SOLV * U] = acc_solv;
      o[ACC_SOLU * U] = acc_solu;
      o[ACC_A0 * U] = acc_a0;
      o[ACC_A1 * U] = acc_a1;
      o[ACC_A2 * U] = acc_a2;
      o[ACC_NPAIR * U] = (double)npair;
    }
  }
  if (cur_s >= 0) reduce_i();
  put_pending();
}

hipError_t launch_tile(const Dev& d, hipStream_t st, const PotConsts& pc, int precision, int schedule,
                       const TileShape& sh, const double* xin) {
  const dim3 G(sh.blocks), B(kBlk);
  const bool sw = pc.inv_w > 0;
  const double fs = fixed_scale(precision);
  if (precision == 0) {
    const Pot<float> P = make_pot<float>(pc);
    if (schedule == 0) {
      if (sw) hipLaunchKernelGGL((k_tile<float, 0, true>), G, B, 0, st, d, P, fs, xin);
      else hipLaunchKernelGGL((k_tile<float, 0, false>), G, B, 0, st, d, P, fs, xin);
    } else {
      if (sw) hipLaunchKernelGGL((k_tile<float, 1, true>), G, B, 0, st, d, P, fs, xin);
      else hipLaunchKernelGGL((k_tile<float, 1, false>), G, B, 0, st, d, P, fs, xin);
    }
  } else {
    const Pot<double> P = make_pot<double>(pc);
    if (schedule == 0) {
      if (sw) hipLaunchKernelGGL((k_tile<double, 0, true>), G, B, 0, st, d, P, fs, xin);
      else hipLaunchKernelGGL((k_tile<double, 0, false>), G, B, 0, st, d, P, fs, xin);
    } else {
      if (sw) hipLaunchKernelGGL((k_tile<double, 1, true>), G, B, 0, st, d, P, fs, xin);
      else hipLaunchKernelGGL((k_tile<double, 1, false>), G, B, 0, st, d, P, fs, xin);
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
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
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
      lbf_switch(l, s.a[0], s.a[1], s.a[2], s.a[3]);
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
  bool moved = false, bad = false;
  for (int a = t; a < d.n_atoms; a += gridDim.x * blockDim.x) {
    // per-atom records written with the slots (zero before the first
    // build; off.w = slot + 1): every load here is independent of the
    // others, and each is needed on every path, so they all go out together
    const double x = pos[3 * a], y = pos[3 * a + 1], z = pos[3 * a + 2];
    const double4 L = d.atom_box[a], off = d.atom_off[a];
    const double xb = d.x_build[3 * a], yb = d.x_build[3 * a + 1], zb = d.x_build[3 * a + 2];
    if (!(isfinite(x) && isfinite(y) && isfinite(z))) bad = true;  // reported; the values still flow
    const double Lk[3] = {L.x, L.y, L.z}, ok[3] = {off.x, off.y, off.z};
    double dd[3] = {x - xb, y - yb, z - zb};
    double r2 = 0;
    for (int k = 0; k < 3; ++k) {
      dd[k] -= Lk[k] * rint(dd[k] / Lk[k]);
      r2 += dd[k] * dd[k];
    }
    // (an atom not yet placed has a zero box: NaN distance, never moved)
    if (r2 > half_skin2) moved = true;
    // (the test reads every component of off, so that its load is not
    // split and the rest of it held back behind the branch)
    const bool placed = off.w > 0.0 && !isnan(off.x + off.y + off.z);
    if (!placed || mode == 2) continue;  // the list build writes the slot data
    const int sl = (int)off.w - 1;
    // Coordinates relative to the atom's SC origin in the image it had at
    // the build (displacement since the build plus the build-time offset),
    // and cleared force accumulators; the charges in .w stay from the
    // build.  If this call rebuilds the list, the build overwrites them for
    // the new slots.
    double q[3];
    for (int k = 0; k < 3; ++k) q[k] = dd[k] + ok[k];
    float* p32 = reinterpret_cast<float*>(d.pos32 + sl);
    double* p64 = reinterpret_cast<double*>(d.pos64 + sl);
    for (int k = 0; k < 3; ++k) {
      p32[k] = (float)q[k];
      p64[k] = q[k];
    }
    const int slots = d.sc_cap * kSc;
    d.ffix[sl] = 0ull;
    d.ffix[slots + sl] = 0ull;
    d.ffix[2 * slots + sl] = 0ull;
  }
  if (bad) atomicOr(d.flags, 4u);
  if (moved && mode != 2) {
    if (mode == 1) __atomic_store_n(d.rebuild, 1, __ATOMIC_RELAXED);
    else atomicOr(d.flags, 2u);
  }
}

// One-wave blocks: the per-atom loads and stores spread over as many
// compute units as there are waves (measured: 0.3 us less per call than
// 256-thread blocks on the 8,973-atom box, with the same kernel duration).
constexpr int kPrepBlk = 64;

hipError_t launch_prepare(const Dev& d, hipStream_t st, const double* pos, const double* lambda, int mode,
                          double half_skin, int schedule) {
  const int g = max(1, min(2048, (max(d.n_atoms, d.n_reps) + kPrepBlk - 1) / kPrepBlk));
  hipLaunchKernelGGL(k_prepare, dim3(g), dim3(kPrepBlk), 0, st, d, pos, lambda, mode, half_skin * half_skin,
                     schedule);
  return hipGetLastError();
}


// Blocks [0, K * kRedChunks): block (k, c) sums chunk c of box k's unit
// partials (fixed chunk bounds; strided per-thread sums, a butterfly per
// wave, the waves in order); the last chunk of box k to
// finish (counter red_done[k]) adds the kRedChunks chunk sums in order and
// writes the energy terms.  Blocks beyond: fixed-point forces -> float64 in
// atom order.
__global__ void __launch_bounds__(kBlk) k_finalize(Dev d, int schedule, double inv_scale, double* __restrict__ terms,
                                                   double* __restrict__ forces, double* __restrict__ dudl,
                                                   long long* __restrict__ n_pairs) {
  __shared__ double red[kBlk / 64][NACC];
  __shared__ int last;
  const int K = d.n_reps;
  const int nred = K * kRedChunks;
  if ((int)blockIdx.x < nred) {
    const int k = blockIdx.x / kRedChunks, c = blockIdx.x % kRedChunks;
    const int u0 = d.rep_ustart[k], u1 = d.rep_ustart[k + 1];
    const int c0 = u0 + (int)((long long)(u1 - u0) * c / kRedChunks);
    const int c1 = u0 + (int)((long long)(u1 - u0) * (c + 1) / kRedChunks);
    const size_t U = (size_t)d.unit_cap;
    double s[NACC] = {0, 0, 0, 0, 0, 0};
    // four units per thread per round, their loads issued together
    for (int u = c0 + threadIdx.x; u < c1; u += 4 * kBlk) {
      double v[4][NACC];
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int j = 0; j < NACC; ++j) v[q][j] = u + q * kBlk < c1 ? d.unit_acc[j * U + u + q * kBlk] : 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int j = 0; j < NACC; ++j) s[j] += v[q][j];
    }
    // a butterfly per wave, then the waves in order
    for (int j = 0; j < NACC; ++j) s[j] = wave_sum(s[j]);
    if ((threadIdx.x & 63) == 0)
      for (int j = 0; j < NACC; ++j) red[threadIdx.x >> 6][j] = s[j];
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int j = 0; j < NACC; ++j) {
        double t = red[0][j];
        for (int w = 1; w < kBlk / 64; ++w) t += red[w][j];
        d.chunk_acc[(size_t)blockIdx.x * NACC + j] = t;
      }
      // publish the chunk sums, then count; the last chunk acquires them all
      last = __hip_atomic_fetch_add(&d.red_done[k], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) ==
             (unsigned int)(kRedChunks - 1);
    }
    __syncthreads();
    if (!last) return;
    // PME partial sums of the box: one slot per thread, a butterfly per
    // wave, the waves in order (the whole block of the box's last chunk)
    __shared__ double pme_red[kBlk / 64][PME_NPART];
    double pme_e[PME_NPART];
    if (d.pme_box) {
      static_assert(kPmeParts == kBlk, "one partial-sum slot per thread");
      const double* pp = d.pme_part + ((size_t)k * kPmeParts + threadIdx.x) * PME_NPART;
#pragma unroll
      for (int j = 0; j < PME_NPART; ++j) pme_e[j] = wave_sum(pp[j]);
      if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int j = 0; j < PME_NPART; ++j) pme_red[threadIdx.x >> 6][j] = pme_e[j];
      __syncthreads();
#pragma unroll
      for (int j = 0; j < PME_NPART; ++j) {
        double t = pme_red[0][j];
        for (int w = 1; w < kBlk / 64; ++w) t += pme_red[w][j];
        pme_e[j] = t;
      }
    }
    if (threadIdx.x != 0) return;
    d.red_done[k] = 0u;
    double a[NACC] = {0, 0, 0, 0, 0, 0};
    for (int q = 0; q < kRedChunks; ++q)
      for (int j = 0; j < NACC; ++j) a[j] += d.chunk_acc[((size_t)k * kRedChunks + q) * NACC + j];
    const double solv = a[ACC_SOLV], solu = a[ACC_SOLU];
    const double a0 = a[ACC_A0], a1 = a[ACC_A1], a2 = a[ACC_A2];
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
    if (d.pme_box) {
      // PME parts of the box (summed above), its self energies, then the
      // background part from the group charges; S-S and W-W join the
      // lambda-independent terms, the S-W part X is scaled like the
      // solute-solvent Coulomb pairs
      const double* e = pme_e;
      const PmeBox B = d.pme_box[k];
      const double bg = -kKe * M_PI / (B.L[0] * B.L[1] * B.L[2] * d.pme_alpha * d.pme_alpha);
      const double* kc = d.pme_const + 4 * (size_t)k;
      const double qs = kc[PME_K_Q_S], qw = kc[PME_K_Q_W];
      const double ss = ((e[PME_E_SS] + e[PME_C_SS]) + kc[PME_K_SELF_S]) + 0.5 * bg * qs * qs;
      const double ww = ((e[PME_E_WW] + e[PME_C_WW]) + kc[PME_K_SELF_W]) + 0.5 * bg * qw * qw;
      const double X = (e[PME_E_SW] + e[PME_C_SW]) + bg * qs * qw;
      t[0] += ww;
      t[1] += ss;
      if (schedule == 0) {
        t[3] += L.a[1] * X;
        t[7] += L.a[3] * X;
      } else {
        t[3] += L.a[0] * X;
        t[4] += X;
        t[7] += L.a[2] * X;
      }
    }
    t[8] = ((t[0] + t[1]) + t[2]) + t[3];
    t[9] = t[6] + t[7];
    if (terms)
      for (int j = 0; j < kNTerms; ++j) terms[k * kNTerms + j] = t[j];
    if (dudl) dudl[k] = t[9];
    d.last_dudl[k] = t[9];
    if (n_pairs) n_pairs[k] = (long long)a[ACC_NPAIR];
    return;
  }
  if (!forces) return;
  // one slot per thread: its three sums and its atom index are independent loads
  const int slots = d.sc_cap * kSc;
  for (int sl = (blockIdx.x - nred) * kBlk + threadIdx.x; sl < slots; sl += (gridDim.x - nred) * kBlk) {
    const int a = d.slot_atom[sl];
    const long long fx = (long long)d.ffix[sl];
    const long long fy = (long long)d.ffix[slots + sl];
    const long long fz = (long long)d.ffix[2 * slots + sl];
    // an empty statement that reads the sums: their loads then go out with
    // the atom index instead of waiting behind the branch on it
    asm volatile("" ::"v"(fx), "v"(fy), "v"(fz));
    if (a >= 0) {
      forces[3 * a] = (double)fx * inv_scale;
      forces[3 * a + 1] = (double)fy * inv_scale;
      forces[3 * a + 2] = (double)fz * inv_scale;
    }
  }
}

hipError_t launch_finalize(const Dev& d, hipStream_t st, int precision, int schedule, double* terms, double* forces,
                           double* dudl, long long* n_pairs) {
  const int gf = forces ? max(1, min(2048, (d.sc_cap * kSc + kBlk - 1) / kBlk)) : 0;
  hipLaunchKernelGGL(k_finalize, dim3(d.n_reps * kRedChunks + gf), dim3(kBlk), 0, st, d, schedule,
                     1.0 / fixed_scale(precision),
                     terms, forces, dudl, n_pairs);
  return hipGetLastError();
}

}  // namespace anb
