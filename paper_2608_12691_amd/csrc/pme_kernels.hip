// Ewald electrostatics by smooth particle-mesh Ewald for the alchemical
// nonbonded path (long-range electrostatics by PME: Simulation Details; the
// smooth PME method of Essmann et al. 1995), with the solute-solvent part
// of the reciprocal energy scaled like the solute-solvent Coulomb pairs
// (Linear Basis Function section, eq. 4).
//
// Per call, after the short-range tile kernel and before the final
// reduction:
//   k_pme_spread    charges -> two int64 fixed-point grids (solute S,
//                   solvent W) with order-n cardinal B-splines, kScSplit
//                   blocks per super-cluster, each over a part of its
//                   slots: their atoms' n^3 points each are summed in an
//                   LDS sub-grid, then added to the grid with one atomic per
//                   point (integer sums: bit-identical from run to run);
//                   further blocks take the excluded pairs' -k_e q q
//                   erf(a r)/r, one thread per pair (the self and charge
//                   parts are constants of the binding);
//   k_pme_fft x2    forward transforms of Z = Q_S + i Q_W along z, then y: a
//                   block per tile of up to 16 adjacent lines in LDS (the z
//                   pass reads and clears the integer grids); mixed-radix
//                   Stockham passes (radices 5, 4, 3, 2); for grids whose
//                   y-z planes fit in LDS, k_pme_fft_yz does both passes,
//                   one block per plane;
//   k_pme_xconv     per tile of x-lines with their mirror lines: forward
//                   transforms along x, the convolution (spectra of Q_S and
//                   Q_W through Z(-m) = conj, the influence function C(m),
//                   the S-S, W-W and S-W energies, G_S + i G_W with
//                   G_S = C (S + c W), G_W = C (W + c S)), inverse transforms
//                   along x;
//   k_pme_fft x2    inverse transforms along y, then z (or k_pme_fft_yz):
//                   the grid then holds the potentials dU/dQ_S (real part)
//                   and dU/dQ_W (imaginary part);
//   k_pme_gather    kScSplit blocks per super-cluster: the sub-grid of the
//                   potential staged in LDS, four threads per atom summing
//                   -q grad(sum_k M M M G) into the fixed-point force sums.
// Energies leave as per-box partial sums in fixed slots; the final
// reduction adds them in order (deterministic).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "anb_kernels.h"

namespace anb {
namespace {

constexpr int kPmeBlk = 256;
// blocks per super-cluster in spreading and gather: block part p takes the
// slots p * 64 / kScSplit .. (p + 1) * 64 / kScSplit - 1 (more blocks than
// compute units for these latency-bound passes)
constexpr int kScSplit = 2;
static_assert(kSc % kScSplit == 0, "equal slot ranges");
constexpr int kTilePts = 1024;  // points of an FFT tile (T(n) lines of n points)
constexpr int kPlaneBlk = 1024; // threads of a y-z plane transform (one block per compute unit by its LDS)
static_assert(kPmeMaxN <= kTilePts, "a tile holds at least one line");

// (no multiply-add contraction in the transforms: every kernel that runs a
// Stockham pass then rounds each product and sum the same way, whatever
// the code around it)
__device__ inline double2 cmul(double2 a, double2 b) {
#pragma clang fp contract(off)
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

// Part `part` of box k's excluded pairs (kPmeParts equal runs), one thread
// per pair: -k_e q_i q_j erf(a r)/r by minimum image and its forces (the
// S-W pairs' scaled by c).  Partial sums into the part's slots.
__device__ inline void pme_corr(const Dev& d, const double* __restrict__ xin, int schedule, double fscale, int k,
                                int part, double (*red)[3]) {
  const PmeBox B = d.pme_box[k];
  const int p0 = B.pair0 + (int)((long long)B.npair * part / kPmeParts);
  const int p1 = B.pair0 + (int)((long long)B.npair * (part + 1) / kPmeParts);
  const double c = lam_c(d.lam[k], schedule);
  const double alpha = d.pme_alpha;
  const double c2a = 2.0 * alpha / sqrt(M_PI);
  const int slots = d.sc_cap * kSc;
  double e[3] = {0.0, 0.0, 0.0};  // S-S, W-W, S-W
  for (int q = p0 + (int)threadIdx.x; q < p1; q += blockDim.x) {
    const PmePair P = d.pme_pairs[q];
    double dv[3], r2 = 0.0;
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      double u = xin[3 * P.j + cc] - xin[3 * P.i + cc];
      u -= B.L[cc] * rint(u / B.L[cc]);
      dv[cc] = u;
      r2 += u * u;
    }
    const double r = sqrt(r2);
    const double er = erf(alpha * r);
    const double v = -P.qq * er / r;
    // dv/dr = -k_e q q [2a/sqrt(pi) exp(-a^2 r^2)/r - erf(a r)/r^2]
    const double dvdr = -P.qq * (c2a * exp(-alpha * alpha * r2) / r - er / r2);
    e[P.kind] += v;
    const double sf = (P.kind == 2 ? c : 1.0) * dvdr / r;
    // F_i = -dv/dx_i = sf d, F_j = -sf d (d = x_j - x_i)
    const int si = d.atom_slot[P.i], sj = d.atom_slot[P.j];
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      add_fixed(d.ffix + (size_t)cc * slots + si, sf * dv[cc], fscale, d.flags);
      add_fixed(d.ffix + (size_t)cc * slots + sj, -sf * dv[cc], fscale, d.flags);
    }
  }
  block_sums<3>(e, red);
  if (threadIdx.x == 0) {
    double* o = d.pme_part + ((size_t)k * kPmeParts + part) * PME_NPART;
    o[PME_C_SS] = e[0];
    o[PME_C_WW] = e[1];
    o[PME_C_SW] = e[2];
  }
}

// ------------------------------------------------- super-cluster sub-grids

// A super-cluster's 64 slots are a compact piece of one box and one group
// (the list build's spatial order): the grid points their splines touch
// form a small block of the grid.  The spreading and the gather of a
// super-cluster work on that block in LDS, so that each of its points costs
// one global access instead of one per atom reaching it.
constexpr int kSubMax = 4096;  // points of a super-cluster's LDS sub-grid at most

// Per-block description of a super-cluster's sub-grid (in LDS).
struct ScSub {
  int k, sol, n;        // box, group (1 = solute), valid slots
  int ref[3];           // grid index of the first valid slot's atom
  int lo[3], ext[3];    // lowest unwrapped offset (spline support included) and extent
  int size;             // ext[0] ext[1] ext[2]
};

__device__ inline int wrap_half(int v, int n) {  // v in (-n, n) -> (-n/2, n/2]
  if (v > n / 2) v -= n;
  else if (v <= -(n + 1) / 2) v += n;
  return v;
}

// Wave 0 reads super-cluster s: per slot its atom, charge, grid offset from
// the reference (unwrapped across the box edge) and spline weights and
// derivatives; then the sub-grid.  All threads return the header (n = 0: empty super-cluster).
template <int N>
__device__ inline void sc_setup(const Dev& d, const double* __restrict__ xin, int s, int part, int* s_atom,
                                int (*s_off)[3], double (*s_th)[3][N], double (*s_dth)[3][N], double* s_q, ScSub& S) {
  if (threadIdx.x < kSc) {
    const int l = threadIdx.x;
    // the slots of this block's part (the others are left empty)
    const int a = l / (kSc / kScSplit) == part ? d.slot_atom[s * kSc + l] : -1;
    const unsigned long long valid = __ballot(a >= 0);
    if (valid == 0) {
      if (l == 0) S.n = 0;
    } else {
      const int first = __builtin_ctzll(valid);
      const int a0 = __builtin_amdgcn_readlane(a, first);
      const int k = d.atom_rep[a0];
      const PmeBox B = d.pme_box[k];
      int off[3] = {0, 0, 0};
      double w[3] = {0.0, 0.0, 0.0};
      int mn[3], mx[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        int i = 0;
        if (a >= 0) i = grid_coord(xin[3 * a + c], B.L[c], B.n[c], w[c]);
        const int ref = __builtin_amdgcn_readlane(i, first);
        off[c] = a >= 0 ? wrap_half(i - ref, B.n[c]) : 0;
        int lo = a >= 0 ? off[c] - (N - 1) : 1 << 30, hi = a >= 0 ? off[c] : -(1 << 30);
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
          lo = min(lo, __shfl_xor(lo, o));
          hi = max(hi, __shfl_xor(hi, o));
        }
        mn[c] = lo;
        mx[c] = hi;
        if (l == 0) S.ref[c] = ref;
      }
      s_atom[l] = a;
      s_q[l] = a >= 0 ? d.type_q[d.atom_type[a]] : 0.0;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        s_off[l][c] = off[c];
        double th[N], dth[N];
        spline_weights<N>(w[c], th, dth);
#pragma unroll
        for (int j = 0; j < N; ++j) {
          s_th[l][c][j] = th[j];
          s_dth[l][c][j] = dth[j];
        }
      }
      if (l == 0) {
        S.k = k;
        S.sol = d.grids[d.atom_grid[a0]].is_solute != 0;
        S.n = __popcll(valid);
        long long size = 1;
        for (int c = 0; c < 3; ++c) {
          S.lo[c] = mn[c];
          S.ext[c] = mx[c] - mn[c] + 1;
          size *= S.ext[c];
        }
        S.size = size <= kSubMax ? (int)size : -1;  // -1: too large for LDS
      }
    }
  }
  __syncthreads();
}

// v mod n for the sub-grid coordinates here, which lie within (-n, 2n): a
// compare and an add (a remainder only outside that range)
__device__ inline int wrap_n(int v, int n) {
  if (v < 0) v += n;
  else if (v >= n) v -= n;
  if (v < 0 || v >= n) {
    v %= n;
    if (v < 0) v += n;
  }
  return v;
}

// Global grid index of sub-grid point (u0, u1, u2).
__device__ inline long long sub_to_grid(const ScSub& S, const PmeBox& B, int u0, int u1, int u2) {
  const int g0 = wrap_n(S.ref[0] + S.lo[0] + u0, B.n[0]);
  const int g1 = wrap_n(S.ref[1] + S.lo[1] + u1, B.n[1]);
  const int g2 = wrap_n(S.ref[2] + S.lo[2] + u2, B.n[2]);
  return ((long long)g0 * B.n[1] + g1) * B.n[2] + g2;
}

// The sub-grid walked by planes: point p = u1 e2 + u2 of the (u1, u2)
// plane has grid offset po within an x-plane and starts at x-plane g0 (the
// walk then steps u0 and wraps g0).
__device__ inline void sub_plane(const ScSub& S, const PmeBox& B, int p, long long& po, int& g0) {
  const int e2 = S.ext[2];
  const int u1 = p / e2, u2 = p - u1 * e2;
  po = (long long)wrap_n(S.ref[1] + S.lo[1] + u1, B.n[1]) * B.n[2] + wrap_n(S.ref[2] + S.lo[2] + u2, B.n[2]);
  g0 = wrap_n(S.ref[0] + S.lo[0], B.n[0]);
}

// Blocks [0, S = kScSplit sc_cap): the spreading of part b % kScSplit of
// super-cluster b / kScSplit: LDS sub-grid, then one global atomic per
// non-zero point (straight global atomics when the sub-grid is too large).
// Blocks beyond: the excluded pairs, part (b - S) % kPmeParts of box
// (b - S) / kPmeParts.
template <int N>
__global__ void __launch_bounds__(kPmeBlk) k_pme_spread(Dev d, const double* __restrict__ xin, int schedule,
                                                        double fscale) {
  if ((int)blockIdx.x >= kScSplit * d.sc_cap) {  // the excluded-pair blocks
    __shared__ double red[kPmeBlk / 64][3];
    const int job = (int)blockIdx.x - kScSplit * d.sc_cap;
    pme_corr(d, xin, schedule, fscale, job / kPmeParts, job % kPmeParts, red);
    return;
  }
  __shared__ int s_atom[kSc];
  __shared__ int s_off[kSc][3];
  __shared__ double s_th[kSc][3][N], s_dth[kSc][3][N];
  __shared__ double s_q[kSc];
  __shared__ ScSub S;
  __shared__ unsigned long long sub[kSubMax];
  const int s = (int)blockIdx.x / kScSplit;
  sc_setup<N>(d, xin, s, (int)blockIdx.x % kScSplit, s_atom, s_off, s_th, s_dth, s_q, S);
  if (S.n == 0) return;
  const PmeBox B = d.pme_box[S.k];
  const bool lds = S.size > 0;
  const int e1 = S.ext[1], e2 = S.ext[2];
  if (lds) {
    for (int e = threadIdx.x; e < S.size; e += blockDim.x) sub[e] = 0ull;
    __syncthreads();
  }
  unsigned long long* grid = d.pme_q + (S.sol ? 0 : d.pme_points) + B.off;
  const double qs = d.pme_qscale;
  for (int idx = threadIdx.x; idx < kSc * N * N; idx += blockDim.x) {
    const int sl = idx / (N * N);
    if (s_atom[sl] < 0) continue;
    const int xy = idx - sl * (N * N);
    const int x = xy / N, y = xy - (xy / N) * N;
    const double wxy = s_q[sl] * qs * s_th[sl][0][x] * s_th[sl][1][y];
    const int u0 = s_off[sl][0] - x - S.lo[0], u1 = s_off[sl][1] - y - S.lo[1];
#pragma unroll
    for (int z = 0; z < N; ++z) {
      const int u2 = s_off[sl][2] - z - S.lo[2];
      const unsigned long long v = (unsigned long long)__double2ll_rn(wxy * s_th[sl][2][z]);
      if (lds) atomicAdd(&sub[((long long)u0 * e1 + u1) * e2 + u2], v);
      else atomicAdd(grid + sub_to_grid(S, B, u0, u1, u2), v);
    }
  }
  if (!lds) return;
  __syncthreads();
  // one global atomic per non-zero point, walked by planes (thread: a point
  // of the (u1, u2) plane, all its u0)
  const int plane = e1 * e2;
  const long long st0 = (long long)B.n[1] * B.n[2];
  for (int p = threadIdx.x; p < plane; p += blockDim.x) {
    long long po;
    int g0;
    sub_plane(S, B, p, po, g0);
    for (int u0 = 0; u0 < S.ext[0]; ++u0) {
      const unsigned long long v = sub[u0 * plane + p];
      if (v != 0ull) atomicAdd(grid + g0 * st0 + po, v);
      g0 = g0 + 1 == B.n[0] ? 0 : g0 + 1;
    }
  }
}

// --------------------------------------------------------------------- FFT

// One Stockham pass of radix R over `lines` lines of n points in LDS
// (point i of line l at l * lstride + i * estride), the butterflies of all
// lines spread over the block.  The R-point DFTs are written out with the
// R-th roots of unity as constants, w = exp(-2 pi i / R) forward and its
// conjugate inverse (sg = -1 / +1 is the sign of the imaginary part):
//   R = 2: y0 = a0 + a1, y1 = a0 - a1;
//   R = 4 (w = sg i): t0 = a0 + a2, t1 = a0 - a2, t2 = a1 + a3,
//     t3 = sg i (a1 - a3); y0 = t0 + t2, y2 = t0 - t2, y1 = t1 + t3,
//     y3 = t1 - t3;
//   R = 3 (w = -1/2 + sg i sin(2 pi/3)): t = a0 - (a1 + a2)/2,
//     u = sg i sin(2 pi/3) (a1 - a2); y0 = a0 + a1 + a2, y1 = t + u, y2 = t - u;
//   R = 5 (w^k = cos(2 pi k/5) + sg i sin(2 pi k/5)): with b1 = a1 + a4,
//     b2 = a2 + a3, d1 = a1 - a4, d2 = a2 - a3, c_k and s_k the cosine and
//     sine of 2 pi k/5: y0 = a0 + b1 + b2; y1, y4 = t1 +- u1 with
//     t1 = a0 + c1 b1 + c2 b2, u1 = sg i (s1 d1 + s2 d2); y2, y3 = t2 +- u2
//     with t2 = a0 + c2 b1 + c1 b2, u2 = sg i (s2 d1 - s1 d2).
template <int R>
__device__ inline void fft_stage(const double2* __restrict__ src, double2* __restrict__ dst, int n, int Ns,
                                 int lines, int lstride, int estride, const double2* __restrict__ W, bool inv) {
#pragma clang fp contract(off)
  const int m = n / R;
  const int step = n / (Ns * R);
  const int total = lines * m;
  const double sg = inv ? 1.0 : -1.0;
  // sg i z
  auto rot = [&](double2 z) { return make_double2(-sg * z.y, sg * z.x); };
  auto add = [](double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); };
  auto sub = [](double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); };
  auto scl = [](double2 a, double c) { return make_double2(a.x * c, a.y * c); };
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    const int line = idx / m, j = idx - line * m;
    const int k = j % Ns;
    const double2* s = src + line * lstride;
    double2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = s[(j + r * m) * estride];
#pragma unroll
    for (int r = 1; r < R; ++r) {
      double2 t = W[r * k * step];
      if (inv) t.y = -t.y;
      v[r] = cmul(v[r], t);
    }
    double2 y[R];
    if constexpr (R == 2) {
      y[0] = add(v[0], v[1]);
      y[1] = sub(v[0], v[1]);
    } else if constexpr (R == 4) {
      const double2 t0 = add(v[0], v[2]), t1 = sub(v[0], v[2]), t2 = add(v[1], v[3]), t3 = rot(sub(v[1], v[3]));
      y[0] = add(t0, t2);
      y[2] = sub(t0, t2);
      y[1] = add(t1, t3);
      y[3] = sub(t1, t3);
    } else if constexpr (R == 3) {
      constexpr double s3 = 0.8660254037844387;  // sin(2 pi/3)
      const double2 b = add(v[1], v[2]);
      const double2 t = sub(v[0], scl(b, 0.5));
      const double2 u = rot(scl(sub(v[1], v[2]), s3));
      y[0] = add(v[0], b);
      y[1] = add(t, u);
      y[2] = sub(t, u);
    } else {
      static_assert(R == 5, "radices 2, 3, 4 and 5");
      constexpr double c1 = 0.30901699437494745, c2 = -0.8090169943749473;  // cos(2 pi/5), cos(4 pi/5)
      constexpr double s1 = 0.9510565162951535, s2 = 0.5877852522924732;    // sin(2 pi/5), sin(4 pi/5)
      const double2 b1 = add(v[1], v[4]), b2 = add(v[2], v[3]);
      const double2 d1 = sub(v[1], v[4]), d2 = sub(v[2], v[3]);
      y[0] = add(add(v[0], b1), b2);
      const double2 t1 = add(add(v[0], scl(b1, c1)), scl(b2, c2));
      const double2 u1 = rot(add(scl(d1, s1), scl(d2, s2)));
      const double2 t2 = add(add(v[0], scl(b1, c2)), scl(b2, c1));
      const double2 u2 = rot(sub(scl(d1, s2), scl(d2, s1)));
      y[1] = add(t1, u1);
      y[4] = sub(t1, u1);
      y[2] = add(t2, u2);
      y[3] = sub(t2, u2);
    }
    double2* o_line = dst + line * lstride;
    const int base = (j / Ns) * Ns * R + k;
#pragma unroll
    for (int q = 0; q < R; ++q) o_line[(base + q * Ns) * estride] = y[q];
  }
}

// Transforms of `lines` lines of n points held in b0 (src = 0) or b1
// (src = 1); the result ends in the one src names after the call (it flips
// with every pass).
__device__ inline void fft_lines(double2* b0, double2* b1, int& src, int n, int lines, int lstride, int estride,
                                 const double2* W, bool inv) {
  int Ns = 1, rem = n;
  while (rem > 1) {
    double2* from = src ? b1 : b0;
    double2* to = src ? b0 : b1;
    int R;
    if (rem % 5 == 0) {
      R = 5;
      fft_stage<5>(from, to, n, Ns, lines, lstride, estride, W, inv);
    } else if (rem % 4 == 0) {
      R = 4;
      fft_stage<4>(from, to, n, Ns, lines, lstride, estride, W, inv);
    } else if (rem % 2 == 0) {
      R = 2;
      fft_stage<2>(from, to, n, Ns, lines, lstride, estride, W, inv);
    } else if (rem % 3 == 0) {
      R = 3;
      fft_stage<3>(from, to, n, Ns, lines, lstride, estride, W, inv);
    } else {
      R = 5;
      fft_stage<5>(from, to, n, Ns, lines, lstride, estride, W, inv);
    }
    Ns *= R;
    rem /= R;
    src ^= 1;
    __syncthreads();
  }
}

// Lines of the pass along `axis` per box: z rows (ix, iy), y columns
// (ix, iz) and x columns (iy, iz), numbered so that consecutive lines are
// adjacent in memory; a block transforms a tile of T(n) consecutive lines.
__device__ inline long long line_addr(int axis, const PmeBox& B, int l, int j) {
  const int n1 = B.n[1], n2 = B.n[2];
  if (axis == 2) return (long long)l * n2 + j;
  const int a = l / n2, iz = l - a * n2;
  if (axis == 1) return ((long long)a * n1 + j) * n2 + iz;
  return ((long long)j * n1 + a) * n2 + iz;
}

// Block t of the pass along `axis` (tiles numbered box by box,
// PmeBox::tiles): its lines staged in LDS (the root table too), the
// Stockham passes, the lines written back; forward (inv = 0) or inverse
// (unnormalised).  first: the lines come from the two integer grids
// (Q_S + i Q_W), which are cleared.  Loads and stores run along the
// memory-contiguous direction (points of a z row; lines of a y or x tile).
__global__ void __launch_bounds__(kPmeBlk) k_pme_fft(Dev d, int axis, int inv, int first) {
  __shared__ double2 b0[kTilePts], b1[kTilePts], W[kPmeMaxN];
  int lo = 0, hi = d.n_reps - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (d.pme_box[mid].tiles[axis] <= (int)blockIdx.x) lo = mid;
    else hi = mid - 1;
  }
  const PmeBox B = d.pme_box[lo];
  // (selects, not a private array indexed at run time, which would live in scratch memory)
  const int n = axis == 0 ? B.n[0] : (axis == 1 ? B.n[1] : B.n[2]);
  const int tab = axis == 0 ? B.tab[0] : (axis == 1 ? B.tab[1] : B.tab[2]);
  const int tile0 = axis == 0 ? B.tiles[0] : (axis == 1 ? B.tiles[1] : B.tiles[2]);
  const int lines = axis == 2 ? B.n[0] * B.n[1] : (axis == 1 ? B.n[0] * B.n[2] : B.n[1] * B.n[2]);
  const int T = tile_lines(n);
  const int l0 = ((int)blockIdx.x - tile0) * T;
  const int nl = min(T, lines - l0);
  for (int e = threadIdx.x; e < n; e += blockDim.x) W[e] = d.pme_roots[tab + e];
  const int np = nl * n;
  double2* g = d.pme_grid + B.off;
  for (int e = threadIdx.x; e < np; e += blockDim.x) {
    const int li = axis == 2 ? e / n : e % nl, j = axis == 2 ? e - li * n : e / nl;
    const long long a = line_addr(axis, B, l0 + li, j);
    double2 v;
    if (first) {
      unsigned long long* qs = d.pme_q + B.off + a;
      unsigned long long* qw = qs + d.pme_points;
      const long long x = (long long)*qs, y = (long long)*qw;
      *qs = 0ull;
      *qw = 0ull;
      const double inv_q = 1.0 / d.pme_qscale;
      v = make_double2((double)x * inv_q, (double)y * inv_q);
    } else {
      v = g[a];
    }
    b0[li * n + j] = v;
  }
  __syncthreads();
  int src = 0;
  fft_lines(b0, b1, src, n, nl, n, 1, W, inv != 0);
  const double2* res = src ? b1 : b0;
  for (int e = threadIdx.x; e < np; e += blockDim.x) {
    const int li = axis == 2 ? e / n : e % nl, j = axis == 2 ? e - li * n : e / nl;
    g[line_addr(axis, B, l0 + li, j)] = res[li * n + j];
  }
}

// The y and z passes of one y-z plane per block, for grids whose planes fit
// in LDS: block (k, ix) (k = blockIdx / max_n0; blocks past box k's x edge
// return) stages plane ix of box k, transforms its z rows and its y columns
// with the passes of the line tiles (forward: z then y, from the integer
// grids, which are cleared; inverse: y then z), and writes it back.  Every
// line receives the same operations as in the line tiles, so the results
// are the same; the two passes take one launch.
__global__ void __launch_bounds__(kPlaneBlk) k_pme_fft_yz(Dev d, int max_n0, int inv) {
  __shared__ double2 b0[kPmePlanePts], b1[kPmePlanePts], W1[kPmeMaxN], W2[kPmeMaxN];
  const int k = (int)blockIdx.x / max_n0, ix = (int)blockIdx.x - k * max_n0;
  const PmeBox B = d.pme_box[k];
  if (ix >= B.n[0]) return;
  const int n1 = B.n[1], n2 = B.n[2], np = n1 * n2;
  for (int e = threadIdx.x; e < n1; e += blockDim.x) W1[e] = d.pme_roots[B.tab[1] + e];
  for (int e = threadIdx.x; e < n2; e += blockDim.x) W2[e] = d.pme_roots[B.tab[2] + e];
  // plane ix: point (iy, iz) at ix n1 n2 + iy n2 + iz
  const long long base = B.off + (long long)ix * np;
  double2* g = d.pme_grid + base;
  for (int e = threadIdx.x; e < np; e += blockDim.x) {
    double2 v;
    if (!inv) {
      unsigned long long* qs = d.pme_q + base + e;
      unsigned long long* qw = qs + d.pme_points;
      const long long x = (long long)*qs, y = (long long)*qw;
      *qs = 0ull;
      *qw = 0ull;
      const double inv_q = 1.0 / d.pme_qscale;
      v = make_double2((double)x * inv_q, (double)y * inv_q);
    } else {
      v = g[e];
    }
    b0[e] = v;
  }
  __syncthreads();
  int src = 0;
  if (!inv) {
    fft_lines(b0, b1, src, n2, n1, n2, 1, W2, false);  // z rows
    fft_lines(b0, b1, src, n1, n2, 1, n2, W1, false);  // y columns
  } else {
    fft_lines(b0, b1, src, n1, n2, 1, n2, W1, true);
    fft_lines(b0, b1, src, n2, n1, n2, 1, W2, true);
  }
  const double2* res = src ? b1 : b0;
  for (int e = threadIdx.x; e < np; e += blockDim.x) g[e] = res[e];
}

// At bind: the influence function C(m) = k_e/(pi V) exp(-pi^2 |m|^2/a^2)/|m|^2
// B(m) of every grid point (C(0) = 0), and per box (block k < K, fixed
// order) the self energies -k_e a/sqrt(pi) sum q^2 of both groups and their
// charges (the background part's input).
__global__ void __launch_bounds__(kPmeBlk) k_pme_init(Dev d) {
  __shared__ double red[kPmeBlk / 64][4];
  for (int k = 0; k < d.n_reps; ++k) {
    const PmeBox B = d.pme_box[k];
    const int n0 = B.n[0], n1 = B.n[1], n2 = B.n[2];
    const long long P = (long long)n0 * n1 * n2;
    const double pref = kKe / (M_PI * B.L[0] * B.L[1] * B.L[2]);
    const double e2 = M_PI * M_PI / (d.pme_alpha * d.pme_alpha);
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < P;
         p += (long long)gridDim.x * blockDim.x) {
      const int i0 = (int)(p / ((long long)n1 * n2));
      const int r = (int)(p - (long long)i0 * n1 * n2);
      const int i1 = r / n2, i2 = r - i1 * n2;
      const int s0 = i0 <= n0 / 2 ? i0 : i0 - n0, s1 = i1 <= n1 / 2 ? i1 : i1 - n1, s2 = i2 <= n2 / 2 ? i2 : i2 - n2;
      const double mx = s0 / B.L[0], my = s1 / B.L[1], mz = s2 / B.L[2];
      const double m2 = mx * mx + my * my + mz * mz;
      d.pme_infl[B.off + p] = p == 0 ? 0.0
                                     : pref * exp(-e2 * m2) / m2 *
                                           (d.pme_bmod[B.tab[0] + i0] * d.pme_bmod[B.tab[1] + i1] *
                                            d.pme_bmod[B.tab[2] + i2]);
    }
  }
  for (int k = blockIdx.x; k < d.n_reps; k += gridDim.x) {
    const ReplicaInfo R = d.reps[k];
    double v[4] = {0.0, 0.0, 0.0, 0.0};  // sum q^2 S, W; sum q S, W
    for (int a = R.atom_off + (int)threadIdx.x; a < R.atom_off + R.n_atoms; a += blockDim.x) {
      const double q = d.type_q[d.atom_type[a]];
      const bool sol = d.grids[d.atom_grid[a]].is_solute != 0;
      v[sol ? 0 : 1] += q * q;
      v[sol ? 2 : 3] += q;
    }
    block_sums<4>(v, red);
    if (threadIdx.x == 0) {
      const double self = -kKe * d.pme_alpha / sqrt(M_PI);
      double* o = d.pme_const + 4 * (size_t)k;
      o[PME_K_SELF_S] = self * v[0];
      o[PME_K_SELF_W] = self * v[1];
      o[PME_K_Q_S] = v[2];
      o[PME_K_Q_W] = v[3];
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------- convolution

// The x-lines (iy, iz) of a box not after their mirror line
// ((-iy) mod n1, (-iz) mod n2) in the order iy n2 + iz: every iz of the rows
// 1 .. (n1-1)/2, then iz <= n2/2 of row 0 and (n1 even) of row n1/2.
__device__ inline void canon_line(int q, int n1, int n2, int& iy, int& iz) {
  const int A = ((n1 - 1) / 2) * n2;
  if (q < A) {
    iy = 1 + q / n2;
    iz = q - (iy - 1) * n2;
    return;
  }
  const int r = q - A, h = n2 / 2 + 1;
  iy = r < h ? 0 : n1 / 2;
  iz = r < h ? r : r - h;
}

// Block (part, box): tiles part, part + kPmeParts, ... of the box's
// canonical x-lines, each tile holding T'(n0) of them with their mirror
// lines in LDS: the forward transforms along x, then for each point m of a
// canonical line with its partner -m on the mirror line (or on the same
// line), the spectra of Q_S and Q_W (Z(-m) = conj), the influence function
// C(m) (table), the S-S, W-W and S-W energies, and G_S + i G_W with
// G_S = C (S + c W), G_W = C (W + c S); then the inverse transforms along x
// and the lines back to HBM.
__global__ void __launch_bounds__(kPmeBlk) k_pme_xconv(Dev d, int schedule) {
  __shared__ double2 b0[kTilePts], b1[kTilePts], W[kPmeMaxN];
  __shared__ double red[kPmeBlk / 64][3];
  const int k = blockIdx.y, part = blockIdx.x;
  const PmeBox B = d.pme_box[k];
  const int n0 = B.n[0], n1 = B.n[1], n2 = B.n[2];
  const int ncanon = canon_lines(n1, n2), TP = pair_tile_lines(n0);
  const int ntiles = (ncanon + TP - 1) / TP;
  const double c = lam_c(d.lam[k], schedule);
  double2* g = d.pme_grid + B.off;
  const double* infl = d.pme_infl + B.off;
  double e[3] = {0.0, 0.0, 0.0};
  if (part < ntiles)
    for (int j = threadIdx.x; j < n0; j += blockDim.x) W[j] = d.pme_roots[B.tab[0] + j];
  for (int t = part; t < ntiles; t += kPmeParts) {
    const int q0 = t * TP, nq = min(TP, ncanon - q0), np = 2 * nq * n0;
    // slot 2i: canonical line q0 + i; slot 2i+1: its mirror line (a copy
    // when the line is its own mirror)
    for (int el = threadIdx.x; el < np; el += blockDim.x) {
      const int slot = el / n0, ix = el - slot * n0;
      int iy, iz;
      canon_line(q0 + (slot >> 1), n1, n2, iy, iz);
      if (slot & 1) {
        iy = iy == 0 ? 0 : n1 - iy;
        iz = iz == 0 ? 0 : n2 - iz;
      }
      b0[el] = g[((long long)ix * n1 + iy) * n2 + iz];
    }
    __syncthreads();
    int src = 0;
    fft_lines(b0, b1, src, n0, 2 * nq, n0, 1, W, false);
    double2* Z = src ? b1 : b0;
    for (int el = threadIdx.x; el < nq * n0; el += blockDim.x) {
      const int i = el / n0, ix = el - i * n0;
      int iy, iz;
      canon_line(q0 + i, n1, n2, iy, iz);
      const int my = iy == 0 ? 0 : n1 - iy, mz = iz == 0 ? 0 : n2 - iz;
      const bool self_line = my == iy && mz == iz;
      const int jx = ix == 0 ? 0 : n0 - ix;
      if (self_line && jx < ix) continue;  // the partner point's thread takes the pair
      const int a = 2 * i * n0 + ix;
      const int b = (self_line ? 2 * i : 2 * i + 1) * n0 + jx;
      const double2 z = Z[a], zc = Z[b];
      const double C = infl[((long long)ix * n1 + iy) * n2 + iz];
      const double2 S = make_double2(0.5 * (z.x + zc.x), 0.5 * (z.y - zc.y));
      const double2 Wv = make_double2(0.5 * (z.y + zc.y), -0.5 * (z.x - zc.x));
      const bool same = a == b;
      const double mult = same ? 1.0 : 2.0;
      e[0] += mult * 0.5 * C * (S.x * S.x + S.y * S.y);
      e[1] += mult * 0.5 * C * (Wv.x * Wv.x + Wv.y * Wv.y);
      e[2] += mult * C * (S.x * Wv.x + S.y * Wv.y);
      const double2 GS = make_double2(C * (S.x + c * Wv.x), C * (S.y + c * Wv.y));
      const double2 GW = make_double2(C * (Wv.x + c * S.x), C * (Wv.y + c * S.y));
      Z[a] = make_double2(GS.x - GW.y, GS.y + GW.x);
      if (!same) Z[b] = make_double2(GS.x + GW.y, GW.x - GS.y);
    }
    __syncthreads();
    fft_lines(b0, b1, src, n0, 2 * nq, n0, 1, W, true);
    const double2* res = src ? b1 : b0;
    for (int el = threadIdx.x; el < np; el += blockDim.x) {
      const int slot = el / n0, ix = el - slot * n0;
      int iy, iz;
      canon_line(q0 + (slot >> 1), n1, n2, iy, iz);
      if (slot & 1) {
        const int my = iy == 0 ? 0 : n1 - iy, mz = iz == 0 ? 0 : n2 - iz;
        if (my == iy && mz == iz) continue;  // the copy of a self-mirrored line
        iy = my;
        iz = mz;
      }
      g[((long long)ix * n1 + iy) * n2 + iz] = res[el];
    }
    __syncthreads();
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

// One block per super-cluster: its sub-grid of the group's potential (G_S
// for a solute super-cluster, G_W otherwise) staged in LDS, then four
// threads per slot: thread p takes the rows (x, y) = p, p + 4, ... (< n^2)
// and sums each z row against the spline weights and their derivatives; the
// three force components are summed over the four threads and added to the
// slot's fixed-point force sums.
template <int N>
__global__ void __launch_bounds__(kPmeBlk) k_pme_gather(Dev d, const double* __restrict__ xin, double fscale) {
  __shared__ int s_atom[kSc];
  __shared__ int s_off[kSc][3];
  __shared__ double s_th[kSc][3][N], s_dth[kSc][3][N];
  __shared__ double s_q[kSc];
  __shared__ ScSub S;
  __shared__ double sub[kSubMax];
  const int s = (int)blockIdx.x / kScSplit;
  sc_setup<N>(d, xin, s, (int)blockIdx.x % kScSplit, s_atom, s_off, s_th, s_dth, s_q, S);
  if (S.n == 0) return;
  const PmeBox B = d.pme_box[S.k];
  const bool lds = S.size > 0;
  const int e1 = S.ext[1], e2 = S.ext[2];
  const double2* grid = d.pme_grid + B.off;
  if (lds) {
    // the group's potential on the sub-grid, walked by planes (thread: a
    // point of the (u1, u2) plane, all its u0), eight loads in flight
    const int plane = e1 * e2;
    const long long st0 = (long long)B.n[1] * B.n[2];
    constexpr int kBatch = 8;
    for (int p = threadIdx.x; p < plane; p += blockDim.x) {
      long long po;
      int g0;
      sub_plane(S, B, p, po, g0);
      for (int u0 = 0; u0 < S.ext[0]; u0 += kBatch) {
        double v[kBatch];
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
          v[k] = 0.0;
          if (u0 + k < S.ext[0]) {
            const double2 g = grid[g0 * st0 + po];
            v[k] = S.sol ? g.x : g.y;
          }
          g0 = g0 + 1 == B.n[0] ? 0 : g0 + 1;
        }
#pragma unroll
        for (int k = 0; k < kBatch; ++k)
          if (u0 + k < S.ext[0]) sub[(u0 + k) * plane + p] = v[k];
      }
    }
    __syncthreads();
  }
  const int slots = d.sc_cap * kSc;
  for (int base = 0; base < kSc * 4; base += blockDim.x) {
    const int t = base + (int)threadIdx.x;
    const int sl = t >> 2, p = t & 3;
    const bool have = sl < kSc && s_atom[sl] >= 0;
    double f0 = 0.0, f1 = 0.0, f2 = 0.0;
    if (have) {
      for (int xy = p; xy < N * N; xy += 4) {
        const int x = xy / N, y = xy - (xy / N) * N;
        const int u0 = s_off[sl][0] - x - S.lo[0], u1 = s_off[sl][1] - y - S.lo[1];
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int z = 0; z < N; ++z) {
          const int u2 = s_off[sl][2] - z - S.lo[2];
          double G;
          if (lds) {
            G = sub[((long long)u0 * e1 + u1) * e2 + u2];
          } else {
            const double2 v = grid[sub_to_grid(S, B, u0, u1, u2)];
            G = S.sol ? v.x : v.y;
          }
          s0 += s_th[sl][2][z] * G;
          s1 += s_dth[sl][2][z] * G;
        }
        const double tx = s_th[sl][0][x], dtx = s_dth[sl][0][x], ty = s_th[sl][1][y], dty = s_dth[sl][1][y];
        f0 += dtx * ty * s0;
        f1 += tx * dty * s0;
        f2 += tx * ty * s1;
      }
    }
    // sum over the slot's four threads (lanes 4m .. 4m+3 of one wave)
#pragma unroll
    for (int o = 1; o <= 2; o <<= 1) {
      f0 += __shfl_xor(f0, o);
      f1 += __shfl_xor(f1, o);
      f2 += __shfl_xor(f2, o);
    }
    if (have && p == 0) {
      const double q = s_q[sl];
      const int gs = s * kSc + sl;
      add_fixed(d.ffix + gs, -q * (B.n[0] / B.L[0]) * f0, fscale, d.flags);
      add_fixed(d.ffix + (size_t)slots + gs, -q * (B.n[1] / B.L[1]) * f1, fscale, d.flags);
      add_fixed(d.ffix + 2 * (size_t)slots + gs, -q * (B.n[2] / B.L[2]) * f2, fscale, d.flags);
    }
  }
}

template <int N>
hipError_t launch_pme_order(const Dev& d, hipStream_t st, const double* pos, int schedule, double fscale,
                            int yz_planes) {
  const dim3 parts(kPmeParts, d.n_reps);
  hipLaunchKernelGGL(k_pme_spread<N>, dim3(kScSplit * d.sc_cap + kPmeParts * d.n_reps), dim3(kPmeBlk), 0, st, d,
                     pos, schedule,
                     fscale);
  const dim3 planes(yz_planes * d.n_reps);
  if (yz_planes > 0) {
    hipLaunchKernelGGL(k_pme_fft_yz, planes, dim3(kPlaneBlk), 0, st, d, yz_planes, 0);
  } else {
    hipLaunchKernelGGL(k_pme_fft, dim3(d.pme_tiles[2]), dim3(kPmeBlk), 0, st, d, 2, 0, 1);
    hipLaunchKernelGGL(k_pme_fft, dim3(d.pme_tiles[1]), dim3(kPmeBlk), 0, st, d, 1, 0, 0);
  }
  hipLaunchKernelGGL(k_pme_xconv, parts, dim3(kPmeBlk), 0, st, d, schedule);
  if (yz_planes > 0) {
    hipLaunchKernelGGL(k_pme_fft_yz, planes, dim3(kPlaneBlk), 0, st, d, yz_planes, 1);
  } else {
    hipLaunchKernelGGL(k_pme_fft, dim3(d.pme_tiles[1]), dim3(kPmeBlk), 0, st, d, 1, 1, 0);
    hipLaunchKernelGGL(k_pme_fft, dim3(d.pme_tiles[2]), dim3(kPmeBlk), 0, st, d, 2, 1, 0);
  }
  hipLaunchKernelGGL(k_pme_gather<N>, dim3(kScSplit * d.sc_cap), dim3(kPmeBlk), 0, st, d, pos, fscale);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_pme(const Dev& d, hipStream_t st, const double* pos, int schedule, int precision, int yz_planes) {
  const double fs = fixed_scale(precision);
  switch (d.pme_order) {
    case 4: return launch_pme_order<4>(d, st, pos, schedule, fs, yz_planes);
    case 5: return launch_pme_order<5>(d, st, pos, schedule, fs, yz_planes);
    case 6: return launch_pme_order<6>(d, st, pos, schedule, fs, yz_planes);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_pme_init(const Dev& d, hipStream_t st) {
  hipLaunchKernelGGL(k_pme_init, dim3(256), dim3(kPmeBlk), 0, st, d);
  return hipGetLastError();
}

}  // namespace anb
