// Ewald electrostatics by smooth particle-mesh Ewald for the alchemical
// nonbonded path (long-range electrostatics by PME: Simulation Details; the
// smooth PME method of Essmann et al. 1995), with the solute-solvent part
// of the reciprocal energy scaled like the solute-solvent Coulomb pairs
// (Linear Basis Function section, eq. 4).
//
// Per call, after the short-range tile kernel and before the final
// reduction:
//   k_pme_spread    charges -> two int64 fixed-point grids (solute S,
//                   solvent W) with order-n cardinal B-splines, one atom per
//                   thread; integer sums, so the grids are bit-identical
//                   from run to run whatever the order of the atomics;
//   k_pme_fft x3    forward complex transform of Z = Q_S + i Q_W, one line
//                   per wave (the first pass reads and clears the integer
//                   grids), mixed-radix 2/3/4/5 Stockham passes in LDS;
//   k_pme_convolve  splits the spectrum into those of Q_S and Q_W through
//                   Z(-m) = conj, multiplies by the influence function C(m),
//                   sums the S-S, W-W and S-W energies and writes
//                   G_S + i G_W with G_S = C (S + c W), G_W = C (W + c S);
//   k_pme_fft x3    inverse transforms: the grid then holds the potentials
//                   dU/dQ_S (real part) and dU/dQ_W (imaginary part);
//   k_pme_gather    per atom the force -q grad(sum_k M M M G), the self part
//                   and the excluded pairs' -k_e q q erf(a r)/r with their
//                   forces, into the fixed-point force sums.
// Energies leave as per-box partial sums in fixed slots; the final
// reduction adds them in order (deterministic).
#include <hip/hip_runtime.h>

#include <cmath>

#include "anb_kernels.h"

namespace anb {
namespace {

constexpr int kPmeBlk = 256;
constexpr int kFftWave = 64;

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Cardinal B-spline weights th[j] = M_N(w + j) and their u-derivatives
// dth[j] = M_{N-1}(w + j) - M_{N-1}(w + j - 1), j < N, for w in [0, 1):
// M_2(w) = w, M_2(w + 1) = 1 - w, then for each order o the recursion
// M_o(u) = [u M_{o-1}(u) + (o - u) M_{o-1}(u - 1)]/(o - 1).
template <int N>
__device__ inline void spline_weights(double w, double (&th)[N], double (&dth)[N]) {
  double m[N];
#pragma unroll
  for (int j = 0; j < N; ++j) m[j] = 0.0;
  m[0] = w;
  m[1] = 1.0 - w;
#pragma unroll
  for (int o = 3; o <= N; ++o) {
    if (o == N) {
      dth[0] = m[0];
#pragma unroll
      for (int j = 1; j < N; ++j) dth[j] = m[j] - m[j - 1];
    }
    const double inv = 1.0 / (o - 1);
#pragma unroll
    for (int j = o - 1; j >= 1; --j) m[j] = ((w + j) * m[j] + (o - w - j) * m[j - 1]) * inv;
    m[0] = w * m[0] * inv;
  }
#pragma unroll
  for (int j = 0; j < N; ++j) th[j] = m[j];
}

// Scaled fractional coordinate of x along an axis of n points and edge L:
// the grid index floor(u) in [0, n) and the fraction w.  A coordinate that
// is not finite or too large to wrap (flagged by the per-call checks) is
// taken as 0, so that every grid index stays in range.
__device__ inline int grid_coord(double x, double L, int n, double& w) {
  double u = x / L * (double)n;
  u -= (double)n * floor(u / (double)n);
  if (!(u >= 0.0 && u < (double)n)) u = 0.0;
  const double f = floor(u);
  w = u - f;
  return (int)f;
}

__device__ inline double lam_c(const LamState& L, int schedule) { return schedule == 0 ? L.a[1] : L.a[0]; }

// Fixed-point add of one force component (round to nearest even); a value
// beyond 2^62 units adds nothing and raises the overflow flag.
__device__ inline void add_fixed(unsigned long long* p, double f, double scale, unsigned int* flags) {
  const double x = f * scale;
  if (!(fabs(x) < 4.611686018427388e18)) {
    atomicOr(flags, 1u);
    return;
  }
  atomicAdd(p, (unsigned long long)__double2ll_rn(x));
}

// Block sum of V values in a fixed order: a butterfly per wave, then the
// waves in order; thread 0 returns the sums.
template <int V>
__device__ inline void block_sums(double (&v)[V], double (*red)[V]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < V; ++j) {
    double x = v[j];
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) x += __shfl_xor(x, s);
    v[j] = x;
  }
  if (lane == 0)
#pragma unroll
    for (int j = 0; j < V; ++j) red[w][j] = v[j];
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < V; ++j) {
      double t = red[0][j];
      for (int q = 1; q < (int)(blockDim.x >> 6); ++q) t += red[q][j];
      v[j] = t;
    }
  }
}

// ---------------------------------------------------------------- spreading

template <int N>
__global__ void __launch_bounds__(kPmeBlk) k_pme_spread(Dev d, const double* __restrict__ xin) {
  for (int a = blockIdx.x * blockDim.x + threadIdx.x; a < d.n_atoms; a += gridDim.x * blockDim.x) {
    const int k = d.atom_rep[a];
    const PmeBox B = d.pme_box[k];
    const double q = d.type_q[d.atom_type[a]];
    const bool sol = d.grids[d.atom_grid[a]].is_solute != 0;
    int i0[3];
    double th[3][N], dth[3][N];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double w;
      i0[c] = grid_coord(xin[3 * a + c], B.L[c], B.n[c], w);
      spline_weights<N>(w, th[c], dth[c]);
    }
    unsigned long long* g = d.pme_q + (sol ? 0 : d.pme_points) + B.off;
    const int n1 = B.n[1], n2 = B.n[2];
#pragma unroll
    for (int x = 0; x < N; ++x) {
      int ix = i0[0] - x;
      ix += ix < 0 ? B.n[0] : 0;
#pragma unroll
      for (int y = 0; y < N; ++y) {
        int iy = i0[1] - y;
        iy += iy < 0 ? n1 : 0;
        const double wxy = q * d.pme_qscale * th[0][x] * th[1][y];
        unsigned long long* row = g + ((long long)ix * n1 + iy) * n2;
#pragma unroll
        for (int z = 0; z < N; ++z) {
          int iz = i0[2] - z;
          iz += iz < 0 ? n2 : 0;
          atomicAdd(row + iz, (unsigned long long)__double2ll_rn(wxy * th[2][z]));
        }
      }
    }
  }
}

// --------------------------------------------------------------------- FFT

// One Stockham pass of radix R over a line of n points in LDS: butterfly j
// (< n/R) reads src[j + r n/R], multiplies by the twiddles
// exp(-+2 pi i r k/(Ns R)) with k = j mod Ns, takes the R-point DFT and
// writes dst[(j/Ns) Ns R + k + q Ns].
template <int R>
__device__ inline void fft_pass(const double2* __restrict__ src, double2* __restrict__ dst, int n, int Ns,
                                const double2* __restrict__ W, bool inv) {
  const int m = n / R;
  const int step = n / (Ns * R);
  for (int j = threadIdx.x; j < m; j += kFftWave) {
    const int k = j % Ns;
    double2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = src[j + r * m];
#pragma unroll
    for (int r = 1; r < R; ++r) {
      double2 t = W[(r * k * step) % n];
      if (inv) t.y = -t.y;
      v[r] = cmul(v[r], t);
    }
    double2 o[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      double2 acc = v[0];
#pragma unroll
      for (int r = 1; r < R; ++r) {
        double2 t = W[((q * r) % R) * m];
        if (inv) t.y = -t.y;
        const double2 p = cmul(v[r], t);
        acc.x += p.x;
        acc.y += p.y;
      }
      o[q] = acc;
    }
    const int base = (j / Ns) * Ns * R + k;
#pragma unroll
    for (int q = 0; q < R; ++q) dst[base + q * Ns] = o[q];
  }
}

// One line per block of one wave: lines of the pass along `axis` are
// numbered box by box (PmeBox::lines); forward (inv = 0) or inverse
// (unnormalised) transform in place.  first: read the line from the two
// integer grids (Q_S + i Q_W) and clear them.
__global__ void __launch_bounds__(kFftWave) k_pme_fft(Dev d, int axis, int inv, int first) {
  __shared__ double2 buf[2][kPmeMaxN];
  const int line = blockIdx.x;
  // the box holding this line (boxes in order, prefix of lines per box)
  int lo = 0, hi = d.n_reps - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (d.pme_box[mid].lines[axis] <= line) lo = mid;
    else hi = mid - 1;
  }
  const PmeBox B = d.pme_box[lo];
  const int l = line - B.lines[axis];
  const int n = B.n[axis], n1 = B.n[1], n2 = B.n[2];
  long long base, stride;
  if (axis == 2) {  // l = ix n1 + iy
    base = (long long)l * n2;
    stride = 1;
  } else if (axis == 1) {  // l = ix n2 + iz
    base = (long long)(l / n2) * n1 * n2 + (l % n2);
    stride = n2;
  } else {  // l = iy n2 + iz
    base = l;
    stride = (long long)n1 * n2;
  }
  double2* g = d.pme_grid + B.off + base;
  if (first) {
    const double inv_q = 1.0 / d.pme_qscale;
    unsigned long long* qs = d.pme_q + B.off + base;
    unsigned long long* qw = qs + d.pme_points;
    for (int j = threadIdx.x; j < n; j += kFftWave) {
      const long long s = (long long)qs[j * stride], w = (long long)qw[j * stride];
      qs[j * stride] = 0ull;
      qw[j * stride] = 0ull;
      buf[0][j] = make_double2((double)s * inv_q, (double)w * inv_q);
    }
  } else {
    for (int j = threadIdx.x; j < n; j += kFftWave) buf[0][j] = g[j * stride];
  }
  __syncthreads();
  const double2* W = d.pme_roots + B.tab[axis];
  int src = 0, Ns = 1, rem = n;
  while (rem > 1) {
    if (rem % 4 == 0) {
      fft_pass<4>(buf[src], buf[src ^ 1], n, Ns, W, inv != 0);
      Ns *= 4;
      rem /= 4;
    } else if (rem % 2 == 0) {
      fft_pass<2>(buf[src], buf[src ^ 1], n, Ns, W, inv != 0);
      Ns *= 2;
      rem /= 2;
    } else if (rem % 3 == 0) {
      fft_pass<3>(buf[src], buf[src ^ 1], n, Ns, W, inv != 0);
      Ns *= 3;
      rem /= 3;
    } else {
      fft_pass<5>(buf[src], buf[src ^ 1], n, Ns, W, inv != 0);
      Ns *= 5;
      rem /= 5;
    }
    src ^= 1;
    __syncthreads();
  }
  for (int j = threadIdx.x; j < n; j += kFftWave) g[j * stride] = buf[src][j];
}

// ------------------------------------------------------------- convolution

__device__ inline int signed_index(int i, int n) { return i <= n / 2 ? i : i - n; }

// Block (part, box): points [P part/kPmeParts, P (part+1)/kPmeParts) of the
// box; each point m with its partner -m handled by the smaller index.
__global__ void __launch_bounds__(kPmeBlk) k_pme_convolve(Dev d, int schedule) {
  __shared__ double red[kPmeBlk / 64][3];
  const int k = blockIdx.y, part = blockIdx.x;
  const PmeBox B = d.pme_box[k];
  const int n0 = B.n[0], n1 = B.n[1], n2 = B.n[2];
  const long long P = (long long)n0 * n1 * n2;
  const long long p0 = P * part / kPmeParts, p1 = P * (part + 1) / kPmeParts;
  const double c = lam_c(d.lam[k], schedule);
  const double V = B.L[0] * B.L[1] * B.L[2];
  const double pref = kKe / (M_PI * V);
  const double e2 = M_PI * M_PI / (d.pme_alpha * d.pme_alpha);
  const double* b0 = d.pme_bmod + B.tab[0];
  const double* b1 = d.pme_bmod + B.tab[1];
  const double* b2 = d.pme_bmod + B.tab[2];
  double2* g = d.pme_grid + B.off;
  double e[3] = {0.0, 0.0, 0.0};
  for (long long p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
    const int i0 = (int)(p / ((long long)n1 * n2));
    const int r = (int)(p - (long long)i0 * n1 * n2);
    const int i1 = r / n2, i2 = r - i1 * n2;
    const int j0 = i0 == 0 ? 0 : n0 - i0, j1 = i1 == 0 ? 0 : n1 - i1, j2 = i2 == 0 ? 0 : n2 - i2;
    const long long pp = ((long long)j0 * n1 + j1) * n2 + j2;
    if (pp < p) continue;  // the partner's thread takes the pair
    const double2 Z = g[p], Zc = g[pp];
    // spectra of Q_S and Q_W at m (both grids are real)
    const double2 S = make_double2(0.5 * (Z.x + Zc.x), 0.5 * (Z.y - Zc.y));
    const double2 Wv = make_double2(0.5 * (Z.y + Zc.y), -0.5 * (Z.x - Zc.x));
    double C = 0.0;
    if (p != 0) {
      const double mx = signed_index(i0, n0) / B.L[0], my = signed_index(i1, n1) / B.L[1],
                   mz = signed_index(i2, n2) / B.L[2];
      const double m2 = mx * mx + my * my + mz * mz;
      C = pref * exp(-e2 * m2) / m2 * (b0[i0] * b1[i1] * b2[i2]);
    }
    const double mult = pp == p ? 1.0 : 2.0;
    e[0] += mult * 0.5 * C * (S.x * S.x + S.y * S.y);
    e[1] += mult * 0.5 * C * (Wv.x * Wv.x + Wv.y * Wv.y);
    e[2] += mult * C * (S.x * Wv.x + S.y * Wv.y);
    const double2 GS = make_double2(C * (S.x + c * Wv.x), C * (S.y + c * Wv.y));
    const double2 GW = make_double2(C * (Wv.x + c * S.x), C * (Wv.y + c * S.y));
    g[p] = make_double2(GS.x - GW.y, GS.y + GW.x);
    if (pp != p) g[pp] = make_double2(GS.x + GW.y, GW.x - GS.y);
  }
  block_sums<3>(e, red);
  if (threadIdx.x == 0) {
    double* o = d.pme_part + ((size_t)k * kPmeParts + part) * PME_NPART;
    o[PME_E_SS] = e[0];
    o[PME_E_WW] = e[1];
    o[PME_E_SW] = e[2];
  }
}

// ------------------------------------------------------------------ gather

// Block (part, box): atoms of the box in kPmeParts equal runs.  The
// reciprocal force of each atom, its self energy and charge, and its
// excluded pairs with later atoms (each pair once), the S-W pairs' forces
// scaled by c.
template <int N>
__global__ void __launch_bounds__(kPmeBlk) k_pme_gather(Dev d, const double* __restrict__ xin, int schedule,
                                                        double fscale) {
  __shared__ double red[kPmeBlk / 64][5];
  const int k = blockIdx.y, part = blockIdx.x;
  const ReplicaInfo R = d.reps[k];
  const PmeBox B = d.pme_box[k];
  const int a0 = R.atom_off + (int)((long long)R.n_atoms * part / kPmeParts);
  const int a1 = R.atom_off + (int)((long long)R.n_atoms * (part + 1) / kPmeParts);
  const double c = lam_c(d.lam[k], schedule);
  const double alpha = d.pme_alpha;
  const double self = -kKe * alpha / sqrt(M_PI);
  const double c2a = 2.0 * alpha / sqrt(M_PI);
  const int slots = d.sc_cap * kSc;
  const int n1 = B.n[1], n2 = B.n[2];
  const double sc[3] = {B.n[0] / B.L[0], B.n[1] / B.L[1], B.n[2] / B.L[2]};
  double e[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // self+excl S-S, W-W, excl S-W, charge S, W
  for (int a = a0 + (int)threadIdx.x; a < a1; a += blockDim.x) {
    const double q = d.type_q[d.atom_type[a]];
    const bool sol = d.grids[d.atom_grid[a]].is_solute != 0;
    const double xa[3] = {xin[3 * a], xin[3 * a + 1], xin[3 * a + 2]};
    int i0[3];
    double th[3][N], dth[3][N];
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      double w;
      i0[cc] = grid_coord(xa[cc], B.L[cc], B.n[cc], w);
      spline_weights<N>(w, th[cc], dth[cc]);
    }
    const double2* g = d.pme_grid + B.off;
    double f[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int x = 0; x < N; ++x) {
      int ix = i0[0] - x;
      ix += ix < 0 ? B.n[0] : 0;
#pragma unroll
      for (int y = 0; y < N; ++y) {
        int iy = i0[1] - y;
        iy += iy < 0 ? n1 : 0;
        const double2* row = g + ((long long)ix * n1 + iy) * n2;
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int z = 0; z < N; ++z) {
          int iz = i0[2] - z;
          iz += iz < 0 ? n2 : 0;
          const double2 v = row[iz];
          const double G = sol ? v.x : v.y;
          s0 += th[2][z] * G;
          s1 += dth[2][z] * G;
        }
        f[0] += dth[0][x] * th[1][y] * s0;
        f[1] += th[0][x] * dth[1][y] * s0;
        f[2] += th[0][x] * th[1][y] * s1;
      }
    }
    double fa[3] = {-q * sc[0] * f[0], -q * sc[1] * f[1], -q * sc[2] * f[2]};
    e[sol ? 0 : 1] += self * q * q;
    e[sol ? 3 : 4] += q;
    // excluded pairs (a, j > a): -k_e q_a q_j erf(a r)/r by minimum image
    for (int x = d.excl_start[a]; x < d.excl_start[a + 1]; ++x) {
      const int j = d.excl_j[x];
      const double qj = d.type_q[d.atom_type[j]];
      const bool solj = d.grids[d.atom_grid[j]].is_solute != 0;
      double dv[3], r2 = 0.0;
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) {
        double t = xin[3 * j + cc] - xa[cc];
        t -= B.L[cc] * rint(t / B.L[cc]);
        dv[cc] = t;
        r2 += t * t;
      }
      const double r = sqrt(r2);
      const double er = erf(alpha * r);
      const double qq = kKe * q * qj;
      const double v = -qq * er / r;
      // dv/dr = -k_e q q [2a/sqrt(pi) exp(-a^2 r^2)/r - erf(a r)/r^2]
      const double dvdr = -qq * (c2a * exp(-alpha * alpha * r2) / r - er / r2);
      const bool cross = sol != solj;
      e[cross ? 2 : (sol ? 0 : 1)] += v;
      const double s = (cross ? c : 1.0) * dvdr / r;
      // F_a = -dv/dx_a = s d, F_j = -s d (d = x_j - x_a)
      const int slj = d.atom_slot[j];
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) {
        fa[cc] += s * dv[cc];
        add_fixed(d.ffix + (size_t)cc * slots + slj, -s * dv[cc], fscale, d.flags);
      }
    }
    const int sl = d.atom_slot[a];
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) add_fixed(d.ffix + (size_t)cc * slots + sl, fa[cc], fscale, d.flags);
  }
  block_sums<5>(e, red);
  if (threadIdx.x == 0) {
    double* o = d.pme_part + ((size_t)k * kPmeParts + part) * PME_NPART;
    o[PME_C_SS] = e[0];
    o[PME_C_WW] = e[1];
    o[PME_C_SW] = e[2];
    o[PME_Q_S] = e[3];
    o[PME_Q_W] = e[4];
  }
}

template <int N>
hipError_t launch_pme_order(const Dev& d, hipStream_t st, const double* pos, int schedule, double fscale) {
  const int gs = max(1, min(2048, (d.n_atoms + kPmeBlk - 1) / kPmeBlk));
  hipLaunchKernelGGL(k_pme_spread<N>, dim3(gs), dim3(kPmeBlk), 0, st, d, pos);
  const int fwd[3] = {2, 1, 0};
  for (int i = 0; i < 3; ++i)
    hipLaunchKernelGGL(k_pme_fft, dim3(d.pme_lines[fwd[i]]), dim3(kFftWave), 0, st, d, fwd[i], 0, i == 0 ? 1 : 0);
  hipLaunchKernelGGL(k_pme_convolve, dim3(kPmeParts, d.n_reps), dim3(kPmeBlk), 0, st, d, schedule);
  for (int i = 2; i >= 0; --i)
    hipLaunchKernelGGL(k_pme_fft, dim3(d.pme_lines[fwd[i]]), dim3(kFftWave), 0, st, d, fwd[i], 1, 0);
  hipLaunchKernelGGL(k_pme_gather<N>, dim3(kPmeParts, d.n_reps), dim3(kPmeBlk), 0, st, d, pos, schedule, fscale);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_pme(const Dev& d, hipStream_t st, const double* pos, int schedule, int precision) {
  const double fs = fixed_scale(precision);
  switch (d.pme_order) {
    case 4: return launch_pme_order<4>(d, st, pos, schedule, fs);
    case 5: return launch_pme_order<5>(d, st, pos, schedule, fs);
    case 6: return launch_pme_order<6>(d, st, pos, schedule, fs);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace anb
