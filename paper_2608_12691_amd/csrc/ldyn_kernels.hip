// Lambda dynamics and d-AFED extended dynamics on the device (FP64).
//
// One launch per MD step, after the nonbonded evaluation (and the dihedral
// CVs when d-AFED is on, or with them: then block K evaluates the CVs and
// their coupling forces itself): block r < K advances replica r's theta,
// block K the auxiliary variables s_k.  The step reads dU/dlambda of the current
// lambda and xi_k of the current positions, and writes the next lambda to
// the array the next evaluation reads, so a whole step (evaluation,
// dihedrals, this update) can be captured in one graph.
//
// Per replica (the paper's extended Hamiltonian, eq. 3 and eqs. 11-14; the
// method's TI, eq. 2):
//   - every `stride` steps a kernel is deposited at theta in both OPES
//     variants (Standard weight exp(U_total/kT), Explore weight 1), merged
//     into the nearest kernel closer than `compress` widths (weight, mean
//     and variance conserved), and rho_bar (the mean of rho_hat over the
//     kernel centres) is recomputed;
//   - U_OPES(theta) = sum over the variants of nu kT ln(rho_hat/rho_bar + eps),
//     F_theta = -dlambda/dtheta dU/dlambda - dU_OPES/dtheta;
//   - dU/dlambda is added to its lambda bin;
//   - theta advances by one BAOAB Langevin step (closing half kick of the
//     previous step, B, A, O with the step's normal deviate, A).
// Auxiliary variables: F_s = kappa wrap(xi - s) (eq. 15), BAOAB at T_s.
// Sums over kernels use fixed-order block reductions (deterministic).
#include <hip/hip_runtime.h>

#include <cmath>

#include "anb_internal.h"
#include "anb_kernels.h"
#include "dihedral_cv.h"

namespace anb {

namespace {

// One wave per block: the kernel sums of a box (at most a few hundred) and
// the CVs reduce without cross-wave barriers (measured: 6.3 against 6.5 us
// per step with the CVs in the launch, 10.5 against 11.3 as two launches).
constexpr int kLdBlk = 64;

__device__ inline double periodic_delta(double a, double b) {
  const double d = a - b;
  return d - 2.0 * floor((d + 1.0) / 2.0);
}
__device__ inline double wrap2(double x) { return x - 2.0 * floor(x / 2.0); }
__device__ inline double wrap_pi(double x) {
  const double y = x - 2.0 * M_PI * floor((x + M_PI) / (2.0 * M_PI));
  return y == -M_PI ? M_PI : y;
}

// Sum of one value per thread of the block, in a fixed order (lanes, then
// waves); every thread gets the result.
__device__ inline double block_sum(double v, double* red) {
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < kLdBlk / 64; ++w) s += red[w];
  __syncthreads();
  return s;
}

// N sums of one value each per thread, reduced together (each in the order
// of block_sum, so each result equals block_sum's); red holds
// kLdBlk / 64 * N doubles.
template <int N>
__device__ inline void block_sums(double (&v)[N], double* red) {
  for (int o = 32; o >= 1; o >>= 1)
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] += __shfl_xor(v[i], o);
  __syncthreads();
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int i = 0; i < N; ++i) red[(threadIdx.x >> 6) * N + i] = v[i];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double s = 0.0;
    for (int w = 0; w < kLdBlk / 64; ++w) s += red[w * N + i];
    v[i] = s;
  }
  __syncthreads();
}

// Minimum of (key, index) over the block; ties to the lower index.
__device__ inline void block_argmin(double key, int idx, double* redk, int* redi, double& out_key, int& out_idx) {
  for (int o = 32; o >= 1; o >>= 1) {
    const double k2 = __shfl_xor(key, o);
    const int i2 = __shfl_xor(idx, o);
    if (k2 < key || (k2 == key && i2 < idx)) {
      key = k2;
      idx = i2;
    }
  }
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    redk[threadIdx.x >> 6] = key;
    redi[threadIdx.x >> 6] = idx;
  }
  __syncthreads();
  out_key = redk[0];
  out_idx = redi[0];
  for (int w = 1; w < kLdBlk / 64; ++w)
    if (redk[w] < out_key || (redk[w] == out_key && redi[w] < out_idx)) {
      out_key = redk[w];
      out_idx = redi[w];
    }
  __syncthreads();
}

struct Kern {
  double* c;
  double* w;
  double* s;
};
__device__ inline Kern kern_of(double* rep, int cap, int variant) {
  double* b = rep + LD_REP_HEADER + 3 * cap * variant;
  return Kern{b, b + cap, b + 2 * cap};
}

// sum_k w_k (s0/s_k) exp(-d^2/2s_k^2) over images -2, 0, +2, and its derivative, one kernel
__device__ inline void kernel_value(double theta, double c, double w, double s, double s0, double& v, double& dv) {
  v = dv = 0.0;
  for (int img = -1; img <= 1; ++img) {
    const double x = theta - c + 2.0 * img;
    const double g = w * (s0 / s) * exp(-0.5 * x * x / (s * s));
    v += g;
    dv += -x / (s * s) * g;
  }
}

// rho_hat numerators, derivatives and total weights of both variants at
// theta, reduced together: p = {v, dv, W} of the Standard kernels, then of
// the Explore kernels
__device__ inline void rho_parts2(const Kern& Ks, int ns, const Kern& Ke, int ne, double s0, double theta,
                                  double* red6, double (&p)[6]) {
#pragma unroll
  for (int i = 0; i < 6; ++i) p[i] = 0.0;
  for (int k = threadIdx.x; k < ns; k += kLdBlk) {
    double g, dg;
    kernel_value(theta, Ks.c[k], Ks.w[k], Ks.s[k], s0, g, dg);
    p[0] += g;
    p[1] += dg;
    p[2] += Ks.w[k];
  }
  for (int k = threadIdx.x; k < ne; k += kLdBlk) {
    double g, dg;
    kernel_value(theta, Ke.c[k], Ke.w[k], Ke.s[k], s0, g, dg);
    p[3] += g;
    p[4] += dg;
    p[5] += Ke.w[k];
  }
  block_sums<6>(p, red6);
}

// mean of rho_hat over the kernel centres
__device__ inline double rho_bar(const Kern& K, int n, double s0, double* red) {
  double W = 0.0;
  for (int k = threadIdx.x; k < n; k += kLdBlk) W += K.w[k];
  W = block_sum(W, red);
  double acc = 0.0;
  for (int k = threadIdx.x; k < n; k += kLdBlk) {
    double r = 0.0;
    for (int j = 0; j < n; ++j) {
      double g, dg;
      kernel_value(K.c[k], K.c[j], K.w[j], K.s[j], s0, g, dg);
      r += g;
    }
    acc += r / W;
  }
  return block_sum(acc, red) / n;
}

// Deposit into one variant: merge into the nearest centre if closer than
// compress * s0, else append.  Returns false when the kernel was dropped
// (capacity reached).
__device__ inline bool deposit_one(const Kern& K, double* count, int cap, double theta, double weight, double s0,
                                   double compress, double* redk, int* redi) {
  const int n = (int)*count;
  bool stored = true;
  if (compress > 0.0 && n > 0) {
    double best = INFINITY;
    int bi = 0x7fffffff;
    for (int k = threadIdx.x; k < n; k += kLdBlk) {
      const double dist = fabs(periodic_delta(theta, K.c[k]));
      if (dist < best || (dist == best && k < bi)) {
        best = dist;
        bi = k;
      }
    }
    double dmin;
    int k;
    block_argmin(best, bi, redk, redi, dmin, k);
    if (dmin < compress * s0) {
      if (threadIdx.x == 0) {
        const double c1 = K.c[k], w1 = K.w[k], s1 = K.s[k];
        const double d = periodic_delta(theta, c1);
        const double w = w1 + weight;
        const double c = c1 + weight * d / w;
        const double var = (w1 * s1 * s1 + weight * s0 * s0) / w + w1 * weight * d * d / (w * w);
        K.c[k] = wrap2(c);
        K.w[k] = w;
        K.s[k] = sqrt(var);
      }
      __syncthreads();
      return true;
    }
  }
  if (threadIdx.x == 0) {
    if (n < cap) {
      K.c[n] = theta;
      K.w[n] = weight;
      K.s[n] = s0;
      *count = (double)(n + 1);
    } else {
      stored = false;
    }
  }
  __syncthreads();
  return stored;
}

}  // namespace

__global__ void __launch_bounds__(kLdBlk) k_ld_step(double* __restrict__ st, const double* __restrict__ dudl,
                                                    const double* __restrict__ xi, const double* __restrict__ noise,
                                                    int noise_rows, double* __restrict__ lam_out,
                                                    unsigned int* __restrict__ flags, LdCv cv) {
  __shared__ double red[kLdBlk / 64];
  __shared__ int redi[kLdBlk / 64];
  __shared__ double red6[kLdBlk / 64 * 6];
  const double* G = st;
  const int K = (int)G[LD_K], n_cv = (int)G[LD_NCV], cap = (int)G[LD_CAP], bins = (int)G[LD_BINS];
  const int stride = (int)G[LD_STRIDE];
  const double kT = G[LD_KT], m = G[LD_MASS], gam = G[LD_GAMMA], h = G[LD_DT];
  const double s0 = G[LD_SIGMA], compress = G[LD_COMPRESS];
  const int width = K + n_cv;  // normal deviates per step
  if ((int)blockIdx.x < K) {
    const int r = blockIdx.x;
    double* R = st + LD_HEADER + (size_t)r * ld_rep_words(cap, bins);
    const long long n = (long long)R[LD_R_N];
    const double* z = noise + (size_t)(n % noise_rows) * width;
    const Kern Ks = kern_of(R, cap, 0), Ke = kern_of(R, cap, 1);
    const double gstd = G[LD_DE_STD] / kT, gexp = G[LD_DE_EXPL] / kT;
    const double nu_s = 1.0 - 1.0 / gstd, nu_e = gexp - 1.0;
    const double eps_s = exp(-gstd / nu_s), eps_e = exp(-gexp / nu_e);
    const double th = R[LD_R_THETA];
    auto bias = [&](double x, double& u, double& du) {
      u = du = 0.0;
      if (R[LD_R_NSTD] <= 0.0) return;
      double q[6];
      rho_parts2(Ks, (int)R[LD_R_NSTD], Ke, (int)R[LD_R_NEXPL], s0, x, red6, q);
      const double as = q[0] / q[2] / R[LD_R_RBAR_STD] + eps_s;
      u += nu_s * kT * log(as);
      du += nu_s * kT * (q[1] / q[2] / R[LD_R_RBAR_STD]) / as;
      const double ae = q[3] / q[5] / R[LD_R_RBAR_EXPL] + eps_e;
      u += nu_e * kT * log(ae);
      du += nu_e * kT * (q[4] / q[5] / R[LD_R_RBAR_EXPL]) / ae;
    };
    if (stride > 0 && n % stride == 0) {
      double u0, du0;
      bias(th, u0, du0);
      bool ok = deposit_one(Ks, R + LD_R_NSTD, cap, th, exp(u0 / kT), s0, compress, red, redi);
      ok = deposit_one(Ke, R + LD_R_NEXPL, cap, th, 1.0, s0, compress, red, redi) && ok;
      if (!ok && threadIdx.x == 0) atomicOr(flags, ALCH_NB_FLAG_LD_CAPACITY);
      const double rs = rho_bar(Ks, (int)R[LD_R_NSTD], s0, red);
      const double re = rho_bar(Ke, (int)R[LD_R_NEXPL], s0, red);
      if (threadIdx.x == 0) {
        R[LD_R_RBAR_STD] = rs;
        R[LD_R_RBAR_EXPL] = re;
      }
      __syncthreads();
    }
    double u, du;
    bias(th, u, du);
    if (threadIdx.x == 0) {
      const bool upper = th > 1.0;
      const double lam = upper ? 2.0 - th : th, dl = upper ? -1.0 : 1.0;
      const double g = dudl[r];
      const double f = -dl * g - du;
      int b = (int)(lam * bins);
      b = b < bins - 1 ? b : bins - 1;
      double* ti = R + LD_REP_HEADER + 6 * cap;
      ti[b] += g;
      ti[bins + b] += 1.0;
      // BAOAB
      double p = R[LD_R_P];
      if (n > 0) p += 0.5 * h * f;
      p += 0.5 * h * f;
      double q = th + 0.5 * h * p / m;
      const double c = exp(-gam * h);
      p = c * p + sqrt((1.0 - c * c) * m * kT) * z[r];
      q += 0.5 * h * p / m;
      q = wrap2(q);
      R[LD_R_P] = p;
      R[LD_R_THETA] = q;
      R[LD_R_LAMBDA] = q > 1.0 ? 2.0 - q : q;
      R[LD_R_LAST_LAMBDA] = lam;
      R[LD_R_DLAM] = dl;
      R[LD_R_U] = u;
      R[LD_R_DU] = du;
      R[LD_R_FTHETA] = f;
      R[LD_R_N] = (double)(n + 1);
      if (lam_out) lam_out[r] = R[LD_R_LAMBDA];
    }
  } else if (n_cv > 0) {
    double* C = st + LD_HEADER + (size_t)K * ld_rep_words(cap, bins);
    const long long n = (long long)C[LD_C_N];
    const double* z = noise + (size_t)(n % noise_rows) * width + K;
    const double kTs = G[LD_KT_S], gs = G[LD_GAMMA_S];
    double* S = C + LD_C_HEADER;
    double* P = S + n_cv;
    const double* M = P + n_cv;
    const double* KA = M + n_cv;
    double* F = S + 4 * n_cv;
    // one BAOAB step of s_k from the CV value xk
    auto advance = [&](int k, double xk) {
      const double s = S[k];
      const double f = KA[k] * wrap_pi(xk - s);
      double p = P[k];
      if (n > 0) p += 0.5 * h * f;
      p += 0.5 * h * f;
      double q = s + 0.5 * h * p / M[k];
      const double c = exp(-gs * h);
      p = c * p + sqrt((1.0 - c * c) * M[k] * kTs) * z[k];
      q += 0.5 * h * p / M[k];
      S[k] = wrap_pi(q);
      P[k] = p;
      F[k] = f;
    };
    if (cv.pos) {
      // the CVs at the current positions, coupled to the current s_k (their
      // forces added to cv.forces); each s_k then advances from its own CV
      // (a CV with an invalid index exerts no force on s_k)
      const dcv::CvOut o{cv.xi_out, nullptr, nullptr, nullptr, cv.u_dafed, cv.forces};
      dcv::cv_block<kLdBlk>(cv.pos, n_cv, cv.idx, S, KA, o, cv.reps, cv.atom_rep, cv.n_atoms, flags,
                            [&](int k, bool ok, double x) { advance(k, ok ? x : S[k]); });
    } else {
      for (int k = threadIdx.x; k < n_cv; k += kLdBlk) advance(k, xi[k]);
    }
    __syncthreads();
    if (threadIdx.x == 0) C[LD_C_N] = (double)(n + 1);
  }
}

__global__ void __launch_bounds__(kLdBlk) k_ld_init(double* __restrict__ st, long long words, LdInit in,
                                                    const double* __restrict__ theta0, const double* __restrict__ s0,
                                                    const double* __restrict__ mass_s,
                                                    const double* __restrict__ kappa) {
  for (long long i = threadIdx.x; i < words; i += kLdBlk) st[i] = 0.0;
  __syncthreads();
  if (threadIdx.x == 0) {
    st[LD_K] = in.K;
    st[LD_NCV] = in.n_cv;
    st[LD_CAP] = in.cap;
    st[LD_BINS] = in.bins;
    st[LD_STRIDE] = in.stride;
    st[LD_KT] = in.kT;
    st[LD_MASS] = in.mass;
    st[LD_GAMMA] = in.gamma;
    st[LD_DT] = in.dt;
    st[LD_SIGMA] = in.sigma;
    st[LD_COMPRESS] = in.compress;
    st[LD_KT_S] = in.kT_s;
    st[LD_GAMMA_S] = in.gamma_s;
    st[LD_DE_STD] = in.de_std;
    st[LD_DE_EXPL] = in.de_expl;
  }
  for (int r = threadIdx.x; r < in.K; r += kLdBlk) {
    double* R = st + LD_HEADER + (size_t)r * ld_rep_words(in.cap, in.bins);
    const double th = wrap2(theta0[r]);
    R[LD_R_THETA] = th;
    R[LD_R_LAMBDA] = th > 1.0 ? 2.0 - th : th;
  }
  if (in.n_cv > 0) {
    double* C = st + LD_HEADER + (size_t)in.K * ld_rep_words(in.cap, in.bins);
    double* S = C + LD_C_HEADER;
    for (int k = threadIdx.x; k < in.n_cv; k += kLdBlk) {
      S[k] = wrap_pi(s0[k]);
      S[2 * in.n_cv + k] = mass_s[k];
      S[3 * in.n_cv + k] = kappa[k];
    }
  }
}

__global__ void k_ld_free_energy(const double* __restrict__ st, double* __restrict__ out) {
  const int K = (int)st[LD_K], cap = (int)st[LD_CAP], bins = (int)st[LD_BINS];
  const int r = blockIdx.x * kLdBlk + threadIdx.x;
  if (r >= K) return;
  const double* ti = st + LD_HEADER + (size_t)r * ld_rep_words(cap, bins) + LD_REP_HEADER + 6 * cap;
  double acc = 0.0;
  bool empty = false;
  for (int b = 0; b < bins; ++b) {
    if (ti[bins + b] <= 0.0) empty = true;
    else acc += ti[b] / ti[bins + b];
  }
  out[r] = empty ? (double)NAN : acc / bins;
}

hipError_t launch_ld_init(hipStream_t st, double* state, long long words, const LdInit& in, const double* theta0,
                          const double* s0, const double* mass_s, const double* kappa) {
  // one block: it clears the whole state, then writes the header and records
  hipLaunchKernelGGL(k_ld_init, dim3(1), dim3(kLdBlk), 0, st, state, words, in, theta0, s0, mass_s, kappa);
  return hipGetLastError();
}

hipError_t launch_ld_step(hipStream_t st, double* state, int K, int n_cv, const double* dudl, const double* xi,
                          const double* noise, int noise_rows, double* lam_out, unsigned int* flags,
                          const LdCv& cv) {
  hipLaunchKernelGGL(k_ld_step, dim3(K + (n_cv > 0 ? 1 : 0)), dim3(kLdBlk), 0, st, state, dudl, xi, noise,
                     noise_rows, lam_out, flags, cv);
  return hipGetLastError();
}

hipError_t launch_ld_free_energy(hipStream_t st, const double* state, int K, double* out) {
  hipLaunchKernelGGL(k_ld_free_energy, dim3((K + kLdBlk - 1) / kLdBlk), dim3(kLdBlk), 0, st, state, out);
  return hipGetLastError();
}

}  // namespace anb
