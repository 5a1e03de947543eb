// Host side of libalchnb: the C ABI declared in include/alch_nb.h.
//
// alch_nb_create() does host-only work (validation, grid planning, list
// capacity); alch_nb_bind() carves a caller-owned device workspace and
// uploads the static tables; every other call enqueues kernels on the bound
// stream and returns without waiting, except those documented as syncing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "alch_nb.h"
#include "anb_internal.h"
#include "anb_kernels.h"

using namespace anb;

namespace {

struct Variant {
  int epu, tiles, blocks;  // entries and tiles (past the first entry) per unit at most, blocks of the launch
};
// Launch variants of the tile kernel searched by alch_nb_autotune().
constexpr Variant kVariants[] = {
    {8, 16, 1024}, {8, 12, 1024}, {8, 24, 1024}, {8, 16, 1280}, {4, 16, 1024}, {8, 64, 1024}, {8, 16, 2048},
};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);
constexpr bool variants_fit() {
  for (const Variant& v : kVariants)
    if (v.epu < 1 || v.epu > kMaxEpu) return false;
  return true;
}
static_assert(ALCH_NB_NTERMS == NTERMS_DEV, "terms per box");
static_assert(variants_fit(), "the tile kernel stages the j-forces of at most kMaxEpu entries per unit");
constexpr int kTimingSlots = 4096;

struct Carve {
  size_t off = 0;
  template <typename T>
  T* take(char* base, size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += sizeof(T) * std::max<size_t>(count, 1);
    return p;
  }
};

}  // namespace

struct alch_nb_ctx {
  // parameters
  alch_nb_params p{};
  std::vector<double> sigma, eps, charge;
  int K = 0, N = 0, G = 0, C = 0, T = 0;
  double r_list = 0;
  // static tables (host copies)
  std::vector<int> atom_type, atom_grid, grid_atoms, excl_start, excl_j, col_grid, atom_rep, atom_comp;
  std::vector<GridInfo> grids;
  std::vector<float4> tp32;
  std::vector<double4> tp64;
  std::vector<float4> dsf32;
  std::vector<ReplicaInfo> reps;
  std::vector<double> sc_box;  // [SC*4]
  int sc_cap = 0, ent_cap = 0, unit_cap = 0;
  size_t ws_bytes = 0;
  // bound state
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  bool bound = false;
  int static_dev = -1;   // device whose library-owned scratch holds the workspace (-1: caller's buffer)
  int fused_blocks = 0;  // blocks of the fused list build (0 = per-phase kernels)
  int fused_possible = 0;  // blocks the fused build may use on this device (0 = not co-resident)
  int list_mode = 0;       // ALCH_NB_LIST_AUTO or ALCH_NB_LIST_PHASES
  Dev dev{};
  PotConsts pc{};
  int variant = 0;
  hipError_t last_hip = hipSuccess;
  unsigned long long* export_counter = nullptr;
  // timing
  int timing_every = 0;      // tile launch of every n-th call timed (0: none)
  long long timing_calls = 0;
  std::vector<hipEvent_t> ev;
  int n_timed = 0;
  double tile_ms = 0;
  long long tile_launches = 0;
  // graph
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  double tuned_ms = 0;  // tile time of the variant chosen by the autotuner
  int ld_ncv = -1;       // auxiliary variables of the last lambda-dynamics state initialised (-1: none)
  bool capturing = false;  // between alch_nb_capture_begin and _end (no timing events then)
  // PME (electrostatics ALCH_NB_ELEC_PME)
  bool pme = false;
  std::vector<PmeBox> pme_box;
  std::vector<double2> pme_roots;
  std::vector<double> pme_bmod;
  long long pme_points = 0;
  int pme_tab = 0;  // entries of the axis tables
  double pme_qscale = 0;  // fixed-point units per e of the charge grids
  int pme_tiles[3] = {0, 0, 0};
  int pme_planes = 0;  // y and z transforms per plane: the largest x edge (0: by line tiles)
  std::vector<PmePair> pme_pairs;
};

static alch_nb_status hip_fail(alch_nb_ctx* c, hipError_t e) {
  if (c) c->last_hip = e;
  return ALCH_NB_E_HIP;
}
#define HIPCHK(call)                          \
  do {                                        \
    hipError_t e_ = (call);                   \
    if (e_ != hipSuccess) return hip_fail(ctx, e_); \
  } while (0)

// A context is usable when bound, and, if bound to the library-owned scratch
// of a device, while no other context has been bound to that scratch since.
static bool is_bound(const alch_nb_ctx* ctx) {
  return ctx->bound && (ctx->static_dev < 0 || anb_static_owns(ctx, ctx->static_dev));
}

// ------------------------------------------------------------------ planning

static void lay_out(alch_nb_ctx* ctx, char* base, Dev* d) {
  Carve cv;
  const size_t N = ctx->N, C = ctx->C, SC = ctx->sc_cap, E = ctx->ent_cap, U = ctx->unit_cap, K = ctx->K;
  const size_t SL = SC * kSc, CL = SC * kScCl;
  d->n_atoms = ctx->N;
  d->n_reps = ctx->K;
  d->n_grids = ctx->G;
  d->n_cols = ctx->C;
  d->sc_cap = ctx->sc_cap;
  d->ent_cap = ctx->ent_cap;
  d->unit_cap = ctx->unit_cap;
  d->n_types = ctx->T;
  d->atom_type = cv.take<int>(base, N);
  d->atom_grid = cv.take<int>(base, N);
  d->atom_rep = cv.take<int>(base, N);
  d->atom_comp = cv.take<int>(base, N);
  d->sc_box = cv.take<double4>(base, SC);
  d->grid_atoms = cv.take<int>(base, N);
  d->grids = cv.take<GridInfo>(base, ctx->G);
  d->reps = cv.take<ReplicaInfo>(base, K);
  d->excl_start = cv.take<int>(base, N + 1);
  d->excl_j = cv.take<int>(base, ctx->excl_j.size());
  d->type_sigma = cv.take<double>(base, ctx->T);
  d->type_eps = cv.take<double>(base, ctx->T);
  d->type_q = cv.take<double>(base, ctx->T);
  d->col_grid = cv.take<int>(base, C);
  d->x_build = cv.take<double>(base, 3 * N);
  d->xw = cv.take<double>(base, 3 * N);
  d->atom_col = cv.take<int>(base, N);
  d->col_count = cv.take<int>(base, C);
  d->col_start = cv.take<int>(base, C);
  d->col_fill = cv.take<int>(base, C);
  d->col_sc = cv.take<int>(base, C);
  d->col_nsc = cv.take<int>(base, C);
  d->bucket = cv.take<int>(base, N);
  d->bucket_z = cv.take<double>(base, N);
  d->sorted = cv.take<int>(base, N);
  d->sc_first = cv.take<int>(base, SC);
  d->sc_n = cv.take<int>(base, SC);
  d->sc_col = cv.take<int>(base, SC);
  d->sc_origin = cv.take<double>(base, 3 * SC);
  d->sc_bbox = cv.take<double>(base, 6 * SC);
  d->cl_bbox = cv.take<double>(base, 6 * CL);
  d->cl_n = cv.take<int>(base, CL);
  d->slot_atom = cv.take<int>(base, SL);
  d->atom_slot = cv.take<int>(base, N);
  d->atom_off = cv.take<double4>(base, N);
  d->atom_box = cv.take<double4>(base, N);
  d->slot_xw = cv.take<double4>(base, SL);
  d->slot_comp = cv.take<int>(base, SL);
  d->slot_type = cv.take<int>(base, SL);
  d->se32 = cv.take<float2>(base, SL);
  d->se64 = cv.take<double2>(base, SL);
  d->q32 = cv.take<float>(base, SL);
  d->q64 = cv.take<double>(base, SL);
  d->sc_ecount = cv.take<int>(base, SC);
  d->sc_estart = cv.take<int>(base, SC);
  d->strip_count = cv.take<int>(base, (size_t)SC * kStrips);
  d->strip_start = cv.take<int>(base, (size_t)SC * kStrips);
  d->sc_ustart = cv.take<int>(base, SC);
  d->ent_jc = cv.take<int>(base, E);
  d->ent_info = cv.take<uint32_t>(base, E);
  d->ent_isc = cv.take<int>(base, E);
  d->ent_mask = cv.take<unsigned long long>(base, E * kScCl);
  d->ent_off = cv.take<double4>(base, E);
  d->units = cv.take<int4>(base, U);
  d->wrec = cv.take<int4>(base, kMaxWaves);
  d->wrec_u0 = cv.take<int4>(base, kMaxWaves);
  d->wrec_jc = cv.take<int>(base, (size_t)kMaxWaves * kMaxEpu);
  d->wrec_info = cv.take<uint32_t>(base, (size_t)kMaxWaves * kMaxEpu);
  d->wrec_off = cv.take<double4>(base, (size_t)kMaxWaves * kMaxEpu);
  d->rep_ustart = cv.take<int>(base, K + 1);
  d->ctr = cv.take<int>(base, 16);
  d->flags = cv.take<unsigned int>(base, 1);
  d->rebuild = cv.take<int>(base, 1);
  d->barrier = cv.take<unsigned int>(base, kBarWords);
  d->pos32 = cv.take<float4>(base, SL);
  d->pos64 = cv.take<double4>(base, SL);
  d->ffix = cv.take<unsigned long long>(base, 3 * SL);
  d->unit_acc = cv.take<double>(base, U * NACC);
  d->chunk_acc = cv.take<double>(base, K * kRedChunks * NACC);
  d->red_done = cv.take<unsigned int>(base, K);
  d->lam = cv.take<LamState>(base, K);
  d->last_dudl = cv.take<double>(base, K);
  d->pg_fix = cv.take<unsigned long long>(base, 3 * SL);
  d->tp32 = cv.take<float4>(base, (size_t)ctx->T * ctx->T);
  d->dsf32 = cv.take<float4>(base, kDsfEntries);
  d->tp64 = cv.take<double4>(base, (size_t)ctx->T * ctx->T);
  d->pot64 = cv.take<double>(base, kPot64Words);
  if (ctx->pme) {
    d->pme_box = cv.take<PmeBox>(base, K);
    d->pme_grid = cv.take<double2>(base, (size_t)ctx->pme_points);
    d->pme_q = cv.take<unsigned long long>(base, 2 * (size_t)ctx->pme_points);
    d->pme_roots = cv.take<double2>(base, ctx->pme_tab);
    d->pme_bmod = cv.take<double>(base, ctx->pme_tab);
    d->pme_part = cv.take<double>(base, K * kPmeParts * PME_NPART);
    d->pme_infl = cv.take<double>(base, (size_t)ctx->pme_points);
    d->pme_const = cv.take<double>(base, 4 * K);
    d->pme_pairs = cv.take<PmePair>(base, ctx->pme_pairs.size());
    d->pme_points = ctx->pme_points;
    for (int a = 0; a < 3; ++a) d->pme_tiles[a] = ctx->pme_tiles[a];
    d->pme_order = ctx->p.pme_order;
    d->pme_alpha = ctx->p.dsf_alpha;
    d->pme_qscale = ctx->pme_qscale;
  } else {
    d->pme_box = nullptr;
    d->pme_grid = nullptr;
    d->pme_q = nullptr;
    d->pme_roots = nullptr;
    d->pme_bmod = nullptr;
    d->pme_part = nullptr;
    d->pme_infl = nullptr;
    d->pme_const = nullptr;
    d->pme_pairs = nullptr;
    d->pme_points = 0;
    d->pme_order = 0;
    d->pme_alpha = 0.0;
    d->pme_qscale = 0.0;
  }
  ctx->export_counter = cv.take<unsigned long long>(base, 1);
  ctx->ws_bytes = cv.off + 256;
}

// Steiner volume of an a x b x c box grown by R.
static double steiner(double a, double b, double c, double R) {
  return a * b * c + 2.0 * (a * b + b * c + c * a) * R + M_PI * (a + b + c) * R * R + 4.0 / 3.0 * M_PI * R * R * R;
}

static std::string tune_key(const alch_nb_ctx* ctx);
static int tune_cache_lookup(const std::string& key);

extern "C" {

// PME grid points along an edge L: the smallest n >= max(L / spacing, 2
// order) whose prime factors are 2, 3 and 5 (-1 beyond kPmeMaxN).
static int pme_size(double L, double spacing, int order) {
  int n = std::max((int)std::ceil(L / spacing - 1e-9), 2 * order);
  for (; n <= kPmeMaxN; ++n) {
    int m = n;
    for (int f : {2, 3, 5})
      while (m % f == 0) m /= f;
    if (m == 1) return n;
  }
  return -1;
}

// Cardinal B-spline M_n(u) (support (0, n)) by its recursion from the hat M_2.
static double bspline_host(double u, int n) {
  if (n == 2) return (u >= 0.0 && u <= 2.0) ? 1.0 - std::fabs(u - 1.0) : 0.0;
  return (u * bspline_host(u, n - 1) + (n - u) * bspline_host(u - 1.0, n - 1)) / (n - 1);
}

// |b(m)|^2 = 1/|sum_{k<n-1} M_n(k+1) exp(2 pi i m k/K)|^2, m < K; a vanishing
// denominator (odd order, m = K/2) takes the mean of its neighbours' |.|^2.
static void bspline_moduli(int K, int n, double* out) {
  std::vector<double> d2(K);
  for (int m = 0; m < K; ++m) {
    double re = 0.0, im = 0.0;
    for (int k = 0; k < n - 1; ++k) {
      const double M = bspline_host(k + 1.0, n);
      const double ph = 2.0 * M_PI * (double)((long long)m * k % K) / K;
      re += M * std::cos(ph);
      im += M * std::sin(ph);
    }
    d2[m] = re * re + im * im;
  }
  for (int m = 0; m < K; ++m)
    if (d2[m] < 1e-10) d2[m] = 0.5 * (d2[(m + K - 1) % K] + d2[(m + 1) % K]);
  for (int m = 0; m < K; ++m) out[m] = 1.0 / d2[m];
}

const char* alch_nb_strerror(alch_nb_status s) {
  switch (s) {
    case ALCH_NB_OK: return "ok";
    case ALCH_NB_E_INVALID_ARG: return "invalid argument";
    case ALCH_NB_E_BOX_TOO_SMALL: return "cutoff + skin exceeds half the shortest box edge";
    case ALCH_NB_E_UNSUPPORTED: return "unsupported request";
    case ALCH_NB_E_CAPACITY: return "neighbour list exceeds its capacity";
    case ALCH_NB_E_HIP: return "HIP runtime error";
    case ALCH_NB_E_NOT_BOUND: return "context has no workspace bound";
    case ALCH_NB_E_NO_DEVICE: return "no usable GPU";
    case ALCH_NB_E_SCRATCH_SIZE: return "workspace larger than the library's static device scratch";
    default: return "unknown status";
  }
}

int32_t alch_nb_num_variants(void) { return kNumVariants; }

double alch_nb_flops_per_pair(int32_t kind) {
  // Work of the defining formulas of one pair, charged per evaluated pair
  // whatever the kernel does to compute them: r^2 5, 1/sqrt(r^2) and r 2,
  // combination rule 3, LJ energy and force 15, switch and its derivative
  // 18, DSF energy and force with erfc evaluated through an exponential 30,
  // force vector and its accumulation 12, energy 2 (87, charged as 90).
  // Solute-solvent pairs add the soft core (x, one reciprocal, dU/dlambda):
  // 30.
  return kind == 0 ? 90.0 : 120.0;
}

alch_nb_status alch_nb_opes_layout(int32_t* offsets, int32_t n) {
  const int32_t v[] = {OPES_THETA, OPES_LAMBDA, OPES_DLAM, OPES_U, OPES_DU, OPES_FTHETA, OPES_KT, OPES_SIGMA,
                       OPES_DE_STD, OPES_DE_EXPL, OPES_N, OPES_CAP, OPES_S_STD, OPES_S_EXPL, OPES_W_STD,
                       OPES_HEADER, OPES_HEADER + OPES_GRID_N, OPES_HEADER + 2 * OPES_GRID_N};
  const int32_t m = (int32_t)(sizeof(v) / sizeof(v[0]));
  if (!offsets || n < m) return ALCH_NB_E_INVALID_ARG;
  for (int i = 0; i < m; ++i) offsets[i] = v[i];
  return ALCH_NB_OK;
}

alch_nb_status alch_nb_create(const alch_nb_params* prm, const alch_nb_system* sys, int32_t n_systems,
                              alch_nb_ctx** out) {
  if (!out) return ALCH_NB_E_INVALID_ARG;
  *out = nullptr;
  if (!prm || !sys || n_systems < 1) return ALCH_NB_E_INVALID_ARG;
  const alch_nb_params& p = *prm;
  if (p.n_types < 1 || !p.sigma || !p.epsilon || !p.charge) return ALCH_NB_E_INVALID_ARG;
  if (!(p.cutoff > 0) || !(p.skin >= 0) || !(p.switch_width >= 0) || !(p.switch_width < p.cutoff) ||
      !(p.dsf_alpha >= 0) || !(p.sc_alpha >= 0))
    return ALCH_NB_E_INVALID_ARG;
  if (p.schedule != ALCH_NB_BEUTLER_DSF && p.schedule != ALCH_NB_LBF_DSF) return ALCH_NB_E_INVALID_ARG;
  if (p.precision != ALCH_NB_FP32_FIXED && p.precision != ALCH_NB_FP64) return ALCH_NB_E_INVALID_ARG;
  if (p.electrostatics != ALCH_NB_ELEC_DSF && p.electrostatics != ALCH_NB_ELEC_PME) return ALCH_NB_E_INVALID_ARG;
  if (p.electrostatics == ALCH_NB_ELEC_PME &&
      (p.pme_order < kPmeMinOrder || p.pme_order > kPmeMaxOrder || !(p.pme_spacing > 0) || !(p.dsf_alpha > 0)))
    return ALCH_NB_E_INVALID_ARG;
  if (p.variant < -1 || p.variant >= kNumVariants) return ALCH_NB_E_INVALID_ARG;
  for (int t = 0; t < p.n_types; ++t)
    if (!(p.sigma[t] > 0) || !(p.epsilon[t] >= 0) || !std::isfinite(p.charge[t])) return ALCH_NB_E_INVALID_ARG;
  if (p.precision == ALCH_NB_FP32_FIXED && p.dsf_alpha * p.cutoff > 4.0) return ALCH_NB_E_UNSUPPORTED;
  const double r_list = p.cutoff + p.skin;
  long long n_total = 0;
  for (int k = 0; k < n_systems; ++k) {
    const alch_nb_system& s = sys[k];
    if (s.n_atoms < 0 || s.n_excl < 0) return ALCH_NB_E_INVALID_ARG;
    if (s.n_atoms > 0 && (!s.type || !s.is_solute)) return ALCH_NB_E_INVALID_ARG;
    if (s.n_excl > 0 && !s.excl) return ALCH_NB_E_INVALID_ARG;
    for (int d = 0; d < 3; ++d)
      if (!(s.box[d] > 0) || !std::isfinite(s.box[d])) return ALCH_NB_E_INVALID_ARG;
    for (int i = 0; i < s.n_atoms; ++i) {
      if (s.type[i] < 0 || s.type[i] >= p.n_types) return ALCH_NB_E_INVALID_ARG;
      if (s.is_solute[i] > 1) return ALCH_NB_E_INVALID_ARG;
    }
    for (int e = 0; e < s.n_excl; ++e) {
      const int i = s.excl[2 * e], j = s.excl[2 * e + 1];
      if (i < 0 || j <= i || j >= s.n_atoms) return ALCH_NB_E_INVALID_ARG;
      if (e > 0) {
        const int pi = s.excl[2 * e - 2], pj = s.excl[2 * e - 1];
        if (i < pi || (i == pi && j <= pj)) return ALCH_NB_E_INVALID_ARG;
      }
    }
    n_total += s.n_atoms;
  }
  if (n_total > (1 << 28)) return ALCH_NB_E_UNSUPPORTED;
  for (int k = 0; k < n_systems; ++k)
    for (int d = 0; d < 3; ++d)
      if (sys[k].n_atoms > 0 && r_list > 0.5 * sys[k].box[d]) return ALCH_NB_E_BOX_TOO_SMALL;

  alch_nb_ctx* ctx = new (std::nothrow) alch_nb_ctx();
  if (!ctx) return ALCH_NB_E_INVALID_ARG;
  ctx->p = p;
  ctx->T = p.n_types;
  ctx->sigma.assign(p.sigma, p.sigma + p.n_types);
  ctx->eps.assign(p.epsilon, p.epsilon + p.n_types);
  ctx->charge.assign(p.charge, p.charge + p.n_types);
  ctx->p.sigma = ctx->sigma.data();
  ctx->p.epsilon = ctx->eps.data();
  ctx->p.charge = ctx->charge.data();
  ctx->K = n_systems;
  ctx->N = (int)n_total;
  ctx->r_list = r_list;
  ctx->variant = p.variant < 0 ? 0 : p.variant;

  // per-atom tables, exclusion CSR (global indices)
  ctx->atom_type.resize(n_total);
  ctx->atom_grid.resize(n_total);
  ctx->atom_rep.resize(n_total);
  ctx->excl_start.assign(n_total + 1, 0);
  {
    int off = 0;
    for (int k = 0; k < n_systems; ++k) {
      const alch_nb_system& s = sys[k];
      for (int i = 0; i < s.n_atoms; ++i) {
        ctx->atom_type[off + i] = s.type[i];
        ctx->atom_rep[off + i] = k;
      }
      for (int e = 0; e < s.n_excl; ++e) ctx->excl_start[off + s.excl[2 * e] + 1]++;
      off += s.n_atoms;
    }
    for (int i = 0; i < ctx->N; ++i) ctx->excl_start[i + 1] += ctx->excl_start[i];
    ctx->excl_j.resize(ctx->excl_start[ctx->N]);
    off = 0;
    std::vector<int> fill(ctx->excl_start.begin(), ctx->excl_start.end() - 1);
    for (int k = 0; k < n_systems; ++k) {
      const alch_nb_system& s = sys[k];
      for (int e = 0; e < s.n_excl; ++e) ctx->excl_j[fill[off + s.excl[2 * e]]++] = off + s.excl[2 * e + 1];
      off += s.n_atoms;
    }
  }

  // connected components of the exclusion graph: atoms in different
  // components are never excluded from each other (fast test in the masks)
  {
    std::vector<int> parent(ctx->N);
    for (int i = 0; i < ctx->N; ++i) parent[i] = i;
    auto find = [&](int x) {
      while (parent[x] != x) {
        parent[x] = parent[parent[x]];
        x = parent[x];
      }
      return x;
    };
    for (int i = 0; i < ctx->N; ++i)
      for (int e = ctx->excl_start[i]; e < ctx->excl_start[i + 1]; ++e) {
        const int a = find(i), b = find(ctx->excl_j[e]);
        if (a != b) parent[std::max(a, b)] = std::min(a, b);
      }
    ctx->atom_comp.resize(ctx->N);
    for (int i = 0; i < ctx->N; ++i) ctx->atom_comp[i] = find(i);
  }

  // grids: per box, the solute group then the environment group
  const double margin = 1.0;  // position jitter allowance in the cluster size estimate
  double ent_est = 0;
  int atom_off = 0, col_base = 0, sc_base = 0;
  for (int k = 0; k < n_systems; ++k) {
    const alch_nb_system& s = sys[k];
    ReplicaInfo rp{};
    for (int d = 0; d < 3; ++d) rp.box[d] = s.box[d];
    rp.atom_off = atom_off;
    rp.n_atoms = s.n_atoms;
    rp.grid0 = (int)ctx->grids.size();
    rp.n_grids = 2;
    rp.sc_begin = sc_base;
    const double V = s.box[0] * s.box[1] * s.box[2];
    const double rho_all = s.n_atoms > 0 ? s.n_atoms / V : 0.0;
    int sc_of_grid[2] = {0, 0};
    double ext[2][3] = {{0, 0, 0}, {0, 0, 0}};
    for (int grp = 1; grp >= 0; --grp) {  // solute (1) first
      GridInfo g{};
      g.replica = k;
      g.is_solute = grp;
      g.atom_off = (int)ctx->grid_atoms.size();
      for (int i = 0; i < s.n_atoms; ++i)
        if ((int)s.is_solute[i] == grp) {
          ctx->grid_atoms.push_back(atom_off + i);
          ctx->atom_grid[atom_off + i] = (int)ctx->grids.size();
        }
      g.n_atoms = (int)ctx->grid_atoms.size() - g.atom_off;
      int ncx = 1, ncy = 1;
      if (g.n_atoms > 512 || (grp == 0 && g.n_atoms > 0)) {
        const double rho = g.n_atoms / V;
        const double b = std::cbrt(kSc / rho);
        ncx = std::max(1, (int)std::floor(s.box[0] / b));
        ncy = std::max(1, (int)std::floor(s.box[1] / b));
        ncx = std::min(ncx, 4096);
        ncy = std::min(ncy, 4096);
      }
      g.ncx = ncx;
      g.ncy = ncy;
      g.wx = s.box[0] / ncx;
      g.wy = s.box[1] / ncy;
      g.col_base = col_base;
      g.sc_base = sc_base;
      g.sc_cap = g.n_atoms > 0 ? (g.n_atoms + kSc - 1) / kSc + ncx * ncy : 0;
      for (int c = 0; c < ncx * ncy; ++c) ctx->col_grid.push_back((int)ctx->grids.size());
      col_base += ncx * ncy;
      sc_base += g.sc_cap;
      sc_of_grid[grp] = g.sc_cap;
      if (g.n_atoms > 0) {
        const double rho = std::max(g.n_atoms / V, 1e-12);
        ext[grp][0] = std::min(g.wx, s.box[0]);
        ext[grp][1] = std::min(g.wy, s.box[1]);
        ext[grp][2] = std::min(s.box[2], kSc / (rho * g.wx * g.wy)) + margin;
      }
      ctx->grids.push_back(g);
    }
    rp.sc_end = sc_base;
    ctx->reps.push_back(rp);
    atom_off += s.n_atoms;
    // entry estimate: j-clusters within r_list of each SC box (cluster
    // density of the whole box), half of them for the half list, full for the
    // solute SCs whose partners all come later
    if (s.n_atoms > 0) {
      const double a_cl = std::cbrt(kCl / rho_all);
      const double R = r_list + 0.9 * a_cl + margin;
      const double rho_cl = rho_all / kCl * 1.25;  // padding allowance
      for (int grp = 0; grp < 2; ++grp) {
        if (sc_of_grid[grp] == 0) continue;
        const double per_sc = rho_cl * steiner(ext[grp][0], ext[grp][1], ext[grp][2], R);
        ent_est += sc_of_grid[grp] * per_sc * (grp == 1 ? 1.0 : 0.5);
      }
    }
  }
  ctx->G = (int)ctx->grids.size();
  ctx->C = (int)ctx->col_grid.size();
  ctx->sc_cap = std::max(1, sc_base);
  ctx->sc_box.assign(4 * (size_t)ctx->sc_cap, 0.0);
  for (const GridInfo& g : ctx->grids)
    for (int s = g.sc_base; s < g.sc_base + g.sc_cap; ++s)
      for (int k = 0; k < 3; ++k) ctx->sc_box[4 * (size_t)s + k] = ctx->reps[g.replica].box[k];
  const double fac = p.list_capacity_factor > 0 ? p.list_capacity_factor : 1.0;
  const double ent_cap = std::ceil(fac * (1.6 * ent_est + 64.0 * ctx->sc_cap + 1024.0));
  if (ent_cap > 2.0e9 / kScCl) {
    delete ctx;
    return ALCH_NB_E_UNSUPPORTED;
  }
  ctx->ent_cap = (int)ent_cap;
  ctx->unit_cap = ctx->ent_cap + ctx->sc_cap + 1;  // a unit holds at least one entry

  // PME grids, root tables and B-spline moduli per box and axis
  if (p.electrostatics == ALCH_NB_ELEC_PME) {
    ctx->pme = true;
    long long pts = 0;
    int tab = 0, tiles[3] = {0, 0, 0};
    int atom0 = 0;
    for (int k = 0; k < n_systems; ++k) {
      PmeBox B{};
      for (int a = 0; a < 3; ++a) {
        B.n[a] = pme_size(sys[k].box[a], p.pme_spacing, p.pme_order);
        B.L[a] = sys[k].box[a];
        if (B.n[a] < 0) {
          delete ctx;
          return ALCH_NB_E_UNSUPPORTED;
        }
      }
      B.off = pts;
      pts += (long long)B.n[0] * B.n[1] * B.n[2];
      const int per_axis[3] = {B.n[1] * B.n[2], B.n[0] * B.n[2], B.n[0] * B.n[1]};
      for (int a = 0; a < 3; ++a) {
        const int T = tile_lines(B.n[a]);
        B.tiles[a] = tiles[a];
        tiles[a] += (per_axis[a] + T - 1) / T;
        B.tab[a] = tab;
        tab += B.n[a];
        for (int i = 0; i < B.n[a]; ++i) {
          const double ph = 2.0 * M_PI * i / B.n[a];
          ctx->pme_roots.push_back(make_double2(std::cos(ph), -std::sin(ph)));
        }
        const size_t b0 = ctx->pme_bmod.size();
        ctx->pme_bmod.resize(b0 + B.n[a]);
        bspline_moduli(B.n[a], p.pme_order, ctx->pme_bmod.data() + b0);
      }
      // excluded pairs of the box: k_e q q and their part
      B.pair0 = (int)ctx->pme_pairs.size();
      for (int e = 0; e < sys[k].n_excl; ++e) {
        const int i = sys[k].excl[2 * e], j = sys[k].excl[2 * e + 1];
        const int si = sys[k].is_solute[i], sj = sys[k].is_solute[j];
        PmePair P{};
        P.i = atom0 + i;
        P.j = atom0 + j;
        P.qq = kKe * p.charge[sys[k].type[i]] * p.charge[sys[k].type[j]];
        P.kind = si && sj ? 0 : (!si && !sj ? 1 : 2);
        ctx->pme_pairs.push_back(P);
      }
      B.npair = (int)ctx->pme_pairs.size() - B.pair0;
      atom0 += sys[k].n_atoms;
      ctx->pme_box.push_back(B);
    }
    if (pts > (1LL << 31)) {
      delete ctx;
      return ALCH_NB_E_UNSUPPORTED;
    }
    ctx->pme_points = pts;
    ctx->pme_tab = tab;
    for (int a = 0; a < 3; ++a) ctx->pme_tiles[a] = tiles[a];
    // one block per y-z plane when every box's plane fits in LDS
    // (ALCHNB_PME_FFT=lines keeps the line tiles)
    {
      int n0max = 0;
      bool fit = true;
      for (const PmeBox& B : ctx->pme_box) {
        n0max = std::max(n0max, B.n[0]);
        fit = fit && (long long)B.n[1] * B.n[2] <= kPmePlanePts;
      }
      const char* env = std::getenv("ALCHNB_PME_FFT");
      ctx->pme_planes = fit && !(env && std::strcmp(env, "lines") == 0) ? n0max : 0;
    }
    // charge-grid scale: a power of two that keeps the largest possible grid
    // value (the box's sum of |q_i|) below 2^62 units, at most 2^52
    double qmax = 1.0;
    for (int k = 0; k < n_systems; ++k) {
      double qs = 0.0;
      for (int i = 0; i < sys[k].n_atoms; ++i) qs += std::fabs(p.charge[sys[k].type[i]]);
      qmax = std::max(qmax, qs);
    }
    ctx->pme_qscale = std::exp2(std::min(52.0, std::floor(62.0 - std::log2(qmax))));
  }

  // potential constants (FP64)
  PotConsts& pc = ctx->pc;
  pc.rc = p.cutoff;
  pc.rc2 = p.cutoff * p.cutoff;
  pc.rs = p.cutoff - p.switch_width;
  pc.inv_w = p.switch_width > 0 ? 1.0 / p.switch_width : 0.0;
  pc.alpha = p.dsf_alpha;
  const double ec = std::erfc(p.dsf_alpha * p.cutoff);
  pc.A = ec / p.cutoff;
  pc.c2a = 2.0 * p.dsf_alpha / std::sqrt(M_PI);
  pc.B = ec / (p.cutoff * p.cutoff) + pc.c2a * std::exp(-p.dsf_alpha * p.dsf_alpha * p.cutoff * p.cutoff) / p.cutoff;
  if (ctx->pme) {  // Ewald real space: erfc(a r)/r with no shift
    pc.A = 0.0;
    pc.B = 0.0;
  }
  pc.sc_alpha = p.sc_alpha;
  // intervals per unit of r: the largest power of two with rc * inv_h <= kDsfN,
  // so that r * inv_h and its fraction are exact in FP32
  pc.inv_h = std::exp2(std::floor(std::log2(kDsfN / p.cutoff)));
  // cubic Hermite pieces, in t = (r - r0)/h as c0 + t (c1 + t (c2 + t c3)),
  // of the smooth factors the FP32 pair math multiplies by q q / r: with
  // f(r) = erfc(a r) and g(r) = (2a/sqrt(pi)) exp(-a^2 r^2) (f' = -g,
  // g' = -2 a^2 r g),
  //   T1(r) = r D(r)          = f - A r + B r (r - rc),  T1' = -g - A + B (2r - rc)
  //   T2(r) = r (-r dD/dr)    = f + r g - B r^2,          T2' = -2 a^2 r^2 g - 2 B r
  // (the shift's cancellation near rc is done here in FP64)
  ctx->dsf32.resize(kDsfEntries);
  {
    const double a = p.dsf_alpha, h = 1.0 / pc.inv_h, A = pc.A, B = pc.B, rc = pc.rc;
    auto f = [&](double r) { return std::erfc(a * r); };
    auto g = [&](double r) { return pc.c2a * std::exp(-a * a * r * r); };
    auto t1 = [&](double r) { return f(r) - A * r + B * r * (r - rc); };
    auto d1 = [&](double r) { return -g(r) - A + B * (2.0 * r - rc); };
    auto t2 = [&](double r) { return f(r) + r * g(r) - B * r * r; };
    auto d2 = [&](double r) { return -2.0 * a * a * r * r * g(r) - 2.0 * B * r; };
    auto piece = [&](double y0, double y1, double d0, double d1) {
      return make_float4((float)y0, (float)(h * d0), (float)(3.0 * (y1 - y0) - h * (2.0 * d0 + d1)),
                         (float)(2.0 * (y0 - y1) + h * (d0 + d1)));
    };
    for (int i = 0; i <= kDsfN; ++i) {
      const double r0 = i * h, r1 = r0 + h;
      ctx->dsf32[2 * i] = piece(t1(r0), t1(r1), d1(r0), d1(r1));
      ctx->dsf32[2 * i + 1] = piece(t2(r0), t2(r1), d2(r0), d2(r1));
    }
  }
  // type-pair table in FP64: sigma_ij, 4 eps_ij, k_e q_i q_j, 1/sigma_ij^6
  ctx->tp32.resize((size_t)ctx->T * ctx->T);
  ctx->tp64.resize((size_t)ctx->T * ctx->T);
  for (int a = 0; a < ctx->T; ++a)
    for (int b = 0; b < ctx->T; ++b) {
      const double sg = 0.5 * (ctx->sigma[a] + ctx->sigma[b]);
      const double e4 = 4.0 * std::sqrt(ctx->eps[a] * ctx->eps[b]);
      const double qq = kKe * ctx->charge[a] * ctx->charge[b];
      const double is6 = 1.0 / (sg * sg * sg * sg * sg * sg);
      ctx->tp64[(size_t)a * ctx->T + b] = make_double4(sg, e4, qq, is6);
      ctx->tp32[(size_t)a * ctx->T + b] = make_float4((float)sg, (float)e4, (float)qq, (float)is6);
    }
  lay_out(ctx, nullptr, &ctx->dev);
  if (p.variant < 0) {
    const int v = tune_cache_lookup(tune_key(ctx));
    if (v >= 0) ctx->variant = v;
  }
  *out = ctx;
  return ALCH_NB_OK;
}

alch_nb_status alch_nb_pme_grid(const alch_nb_ctx* ctx, int32_t k, int32_t dims[3]) {
  if (!ctx || !dims || k < 0 || k >= ctx->K) return ALCH_NB_E_INVALID_ARG;
  if (!ctx->pme) return ALCH_NB_E_UNSUPPORTED;
  for (int a = 0; a < 3; ++a) dims[a] = ctx->pme_box[k].n[a];
  return ALCH_NB_OK;
}

alch_nb_status alch_nb_workspace_size(const alch_nb_ctx* ctx, size_t* bytes) {
  if (!ctx || !bytes) return ALCH_NB_E_INVALID_ARG;
  *bytes = ctx->ws_bytes;
  return ALCH_NB_OK;
}

static void destroy_graph(alch_nb_ctx* ctx) {
  if (ctx->gexec) hipGraphExecDestroy(ctx->gexec);
  if (ctx->graph) hipGraphDestroy(ctx->graph);
  ctx->gexec = nullptr;
  ctx->graph = nullptr;
}

alch_nb_status alch_nb_bind(alch_nb_ctx* ctx, void* d_ws, size_t bytes, void* stream) {
  if (!ctx || !d_ws) return ALCH_NB_E_INVALID_ARG;
  if (ctx->static_dev >= 0) anb_static_release(ctx);
  return anb_bind(ctx, d_ws, bytes, stream, -1);
}

}  // extern "C"

// Bind to device memory: the caller's buffer (static_device < 0) or the
// library-owned scratch of a device.  Clears the workspace, uploads the
// static tables and waits for the uploads; allocates nothing.
alch_nb_status anb_bind(alch_nb_ctx* ctx, void* d_ws, size_t bytes, void* stream, int static_device) {
  if (!ctx || !d_ws) return ALCH_NB_E_INVALID_ARG;
  if (bytes < ctx->ws_bytes || (reinterpret_cast<uintptr_t>(d_ws) & 255u)) return ALCH_NB_E_INVALID_ARG;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return ALCH_NB_E_NO_DEVICE;
  ctx->bound = false;
  ctx->static_dev = static_device;
  destroy_graph(ctx);
  ctx->ws = reinterpret_cast<char*>(d_ws);
  ctx->stream = reinterpret_cast<hipStream_t>(stream);
  lay_out(ctx, ctx->ws, &ctx->dev);
  Dev& d = ctx->dev;
  hipStream_t st = ctx->stream;
  // every index table starts valid (zero) so that no phase can read garbage
  HIPCHK(hipMemsetAsync(ctx->ws, 0, ctx->ws_bytes, st));
  {
    int dev_id = 0, n_cu = 0;
    HIPCHK(hipGetDevice(&dev_id));
    HIPCHK(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev_id));
    const int per_cu = list_fused_max_blocks();
    const char* env = std::getenv("ALCHNB_LIST_KERNELS");
    if (env && std::strcmp(env, "split") == 0) ctx->list_mode = ALCH_NB_LIST_PHASES;
    ctx->fused_possible = (per_cu >= 1 && n_cu > 0) ? n_cu : 0;  // one block of 8 waves per CU
    ctx->fused_blocks = ctx->list_mode == ALCH_NB_LIST_PHASES ? 0 : ctx->fused_possible;
  }
  auto up = [&](const void* dst, const void* src, size_t n) -> hipError_t {
    if (n == 0) return hipSuccess;
    return hipMemcpyAsync(const_cast<void*>(dst), src, n, hipMemcpyHostToDevice, st);
  };
  HIPCHK(up(d.atom_type, ctx->atom_type.data(), sizeof(int) * ctx->N));
  HIPCHK(up(d.atom_grid, ctx->atom_grid.data(), sizeof(int) * ctx->N));
  HIPCHK(up(d.atom_rep, ctx->atom_rep.data(), sizeof(int) * ctx->N));
  HIPCHK(up(d.atom_comp, ctx->atom_comp.data(), sizeof(int) * ctx->N));
  HIPCHK(up(d.sc_box, ctx->sc_box.data(), sizeof(double) * ctx->sc_box.size()));
  HIPCHK(up(d.grid_atoms, ctx->grid_atoms.data(), sizeof(int) * ctx->grid_atoms.size()));
  HIPCHK(up(d.grids, ctx->grids.data(), sizeof(GridInfo) * ctx->G));
  HIPCHK(up(d.reps, ctx->reps.data(), sizeof(ReplicaInfo) * ctx->K));
  HIPCHK(up(d.excl_start, ctx->excl_start.data(), sizeof(int) * (ctx->N + 1)));
  HIPCHK(up(d.excl_j, ctx->excl_j.data(), sizeof(int) * ctx->excl_j.size()));
  HIPCHK(up(d.type_sigma, ctx->sigma.data(), sizeof(double) * ctx->T));
  HIPCHK(up(d.type_eps, ctx->eps.data(), sizeof(double) * ctx->T));
  HIPCHK(up(d.type_q, ctx->charge.data(), sizeof(double) * ctx->T));
  HIPCHK(up(d.col_grid, ctx->col_grid.data(), sizeof(int) * ctx->C));
  HIPCHK(up(d.tp32, ctx->tp32.data(), sizeof(float4) * ctx->tp32.size()));
  HIPCHK(up(d.dsf32, ctx->dsf32.data(), sizeof(float4) * ctx->dsf32.size()));
  HIPCHK(up(d.tp64, ctx->tp64.data(), sizeof(double4) * ctx->tp64.size()));
  double pw[kPot64Words];
  pot64_words(ctx->pc, pw);
  HIPCHK(up(d.pot64, pw, sizeof(pw)));
  if (ctx->pme) {
    HIPCHK(up(d.pme_box, ctx->pme_box.data(), sizeof(PmeBox) * ctx->pme_box.size()));
    HIPCHK(up(d.pme_pairs, ctx->pme_pairs.data(), sizeof(PmePair) * ctx->pme_pairs.size()));
    HIPCHK(up(d.pme_roots, ctx->pme_roots.data(), sizeof(double2) * ctx->pme_roots.size()));
    HIPCHK(up(d.pme_bmod, ctx->pme_bmod.data(), sizeof(double) * ctx->pme_bmod.size()));
    HIPCHK(launch_pme_init(d, st));
  }
  HIPCHK(launch_init(d, st));
  // the host copies must outlive the asynchronous uploads
  HIPCHK(hipStreamSynchronize(st));
  ctx->n_timed = 0;
  ctx->bound = true;
  return ALCH_NB_OK;
}

extern "C" {

static TileShape shape_of(const alch_nb_ctx* ctx) {
  const Variant& v = kVariants[ctx->variant];
  TileShape s;
  s.epu = v.epu;
  s.tiles = v.tiles;
  const long long need = ((long long)ctx->unit_cap + 3) / 4;
  long long b = std::min<long long>(v.blocks, std::max<long long>(8, need));
  b = std::min<long long>((b + 7) / 8 * 8, kMaxWaves / 4);
  s.blocks = (int)b;
  return s;
}

static alch_nb_status enqueue_compute(alch_nb_ctx* ctx, const double* pos, const double* lam, uint32_t flags,
                                      const alch_nb_out* out, bool allow_timing) {
  const alch_nb_params& p = ctx->p;
  int mode = 0;
  if (flags & ALCH_NB_FORCE_REBUILD) mode = 2;
  else if (flags & ALCH_NB_AUTO_REBUILD) mode = p.skin > 0 ? 1 : 2;
  const TileShape sh = shape_of(ctx);
  const Dev& d = ctx->dev;
  hipStream_t st = ctx->stream;
  HIPCHK(launch_prepare(d, st, pos, lam, mode, 0.5 * p.skin, p.schedule));
  HIPCHK(launch_list_build(d, st, pos, ctx->r_list, sh, ctx->fused_blocks));
  const bool timed = allow_timing && ctx->timing_every > 0 && (ctx->timing_calls++ % ctx->timing_every) == 0 &&
                     ctx->n_timed < kTimingSlots;
  if (timed) HIPCHK(hipEventRecord(ctx->ev[2 * ctx->n_timed], st));
  HIPCHK(launch_tile(d, st, ctx->pc, p.precision, p.schedule, sh, pos));
  if (timed) {
    HIPCHK(hipEventRecord(ctx->ev[2 * ctx->n_timed + 1], st));
    ctx->n_timed++;
  }
  if (ctx->pme) HIPCHK(launch_pme(d, st, pos, p.schedule, p.precision, ctx->pme_planes));
  HIPCHK(launch_finalize(d, st, p.precision, p.schedule, out ? out->terms : nullptr, out ? out->forces : nullptr,
                         out ? out->dudl : nullptr, out ? reinterpret_cast<long long*>(out->n_pairs) : nullptr));
  return ALCH_NB_OK;
}

alch_nb_status alch_nb_compute(alch_nb_ctx* ctx, const double* d_pos, const double* d_lambda, uint32_t flags,
                               const alch_nb_out* out) {
  if (!ctx) return ALCH_NB_E_INVALID_ARG;
  if (!is_bound(ctx)) return ALCH_NB_E_NOT_BOUND;
  if (!d_pos || !d_lambda) return ALCH_NB_E_INVALID_ARG;
  return enqueue_compute(ctx, d_pos, d_lambda, flags, out, !ctx->capturing);
}

alch_nb_status alch_nb_build_list(alch_nb_ctx* ctx, const double* d_pos) {
  if (!ctx) return ALCH_NB_E_INVALID_ARG;
  if (!is_bound(ctx)) return ALCH_NB_E_NOT_BOUND;
  if (!d_pos) return ALCH_NB_E_INVALID_ARG;
  const Dev& d = ctx->dev;
  HIPCHK(launch_prepare(d, ctx->stream, d_pos, nullptr, 2, 0.5 * ctx->p.skin, ctx->p.schedule));
  HIPCHK(launch_list_build(d, ctx->stream, d_pos, ctx->r_list, shape_of(ctx), ctx->fused_blocks));
  return ALCH_NB_OK;
}

alch_nb_status alch_nb_set_variant(alch_nb_ctx* ctx, int32_t variant) {
  if (!ctx || variant < 0 || variant >= kNumVariants) return ALCH_NB_E_INVALID_ARG;
  ctx->variant = variant;
  destroy_graph(ctx);
  if (ctx->bound) HIPCHK(launch_units(ctx->dev, ctx->stream, shape_of(ctx)));  // units of this shape
  return ALCH_NB_OK;
}

alch_nb_status alch_nb_set_list_mode(alch_nb_ctx* ctx, int32_t mode) {
  if (!ctx || (mode != ALCH_NB_LIST_AUTO && mode != ALCH_NB_LIST_PHASES)) return ALCH_NB_E_INVALID_ARG;
  ctx->list_mode = mode;
  ctx->fused_blocks = mode == ALCH_NB_LIST_PHASES ? 0 : ctx->fused_possible;
  destroy_graph(ctx);  // a captured step holds the old launches
  return ALCH_NB_OK;
}

int32_t alch_nb_get_list_mode(const alch_nb_ctx* ctx) {
  if (!ctx) return -1;
  return ctx->fused_blocks > 0 ? ALCH_NB_LIST_FUSED_ACTIVE : ALCH_NB_LIST_PHASES;
}

alch_nb_status alch_nb_set_timing(alch_nb_ctx* ctx, int32_t every) {
  if (!ctx || every < 0) return ALCH_NB_E_INVALID_ARG;
  if (every > 0 && ctx->ev.empty()) {
    // created on first use, so that binding creates no HIP objects
    ctx->ev.resize(2 * kTimingSlots);
    for (auto& e : ctx->ev) HIPCHK(hipEventCreate(&e));
  }
  ctx->timing_every = every;
  ctx->timing_calls = 0;
  return ALCH_NB_OK;
}

static alch_nb_status collect_timing(alch_nb_ctx* ctx) {
  for (int i = 0; i < ctx->n_timed; ++i) {
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, ctx->ev[2 * i], ctx->ev[2 * i + 1]));
    ctx->tile_ms += ms;
    ctx->tile_launches++;
  }
  ctx->n_timed = 0;
  return ALCH_NB_OK;
}

alch_nb_status alch_nb_get_flags(alch_nb_ctx* ctx, uint32_t* flags) {
  if (!ctx || !flags) return ALCH_NB_E_INVALID_ARG;
  if (!is_bound(ctx)) return ALCH_NB_E_NOT_BOUND;
  unsigned int f = 0;
  HIPCHK(hipMemcpyAsync(&f, ctx->dev.flags, sizeof(f), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  HIPCHK(hipMemsetAsync(ctx->dev.flags, 0, sizeof(unsigned int), ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  *flags = f;
  return ALCH_NB_OK;
}

alch_nb_status alch_nb_get_stats(alch_nb_ctx* ctx, alch_nb_stats* s) {
  if (!ctx || !s) return ALCH_NB_E_INVALID_ARG;
  std::memset(s, 0, sizeof(*s));
  s->n_atoms = ctx->N;
  s->n_systems = ctx->K;
  s->entry_capacity = ctx->ent_cap;
  s->unit_capacity = ctx->unit_cap;
  s->variant = ctx->variant;
  const TileShape sh = shape_of(ctx);
  s->entries_per_unit = sh.epu;
  s->blocks = sh.blocks;
  if (!ctx->bound) return ALCH_NB_OK;
  int c[16];
  HIPCHK(hipMemcpyAsync(c, ctx->dev.ctr, sizeof(c), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  alch_nb_status r = collect_timing(ctx);
  if (r != ALCH_NB_OK) return r;
  s->n_entries = c[CTR_ENT_NEED];
  s->n_units = c[CTR_UNIT_NEED];
  s->n_rebuilds = c[CTR_NBUILD];
  s->n_tiles = c[CTR_TILES];
  s->n_superclusters = ctx->sc_cap;
  s->tile_ms_total = ctx->tile_ms;
  s->tile_launches_timed = ctx->tile_launches;
  return ALCH_NB_OK;
}

alch_nb_status alch_nb_export_pairs(alch_nb_ctx* ctx, int32_t* d_pairs, int64_t cap, int64_t* n_out) {
  if (!ctx || !n_out || cap < 0 || (cap > 0 && !d_pairs)) return ALCH_NB_E_INVALID_ARG;
  if (!is_bound(ctx)) return ALCH_NB_E_NOT_BOUND;
  HIPCHK(hipMemsetAsync(ctx->export_counter, 0, sizeof(unsigned long long), ctx->stream));
  HIPCHK(launch_export(ctx->dev, ctx->stream, ctx->r_list, d_pairs, cap, ctx->export_counter));
  unsigned long long n = 0;
  HIPCHK(hipMemcpyAsync(&n, ctx->export_counter, sizeof(n), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  *n_out = (int64_t)n;
  return (int64_t)n > cap ? ALCH_NB_E_CAPACITY : ALCH_NB_OK;
}

alch_nb_status alch_nb_capture_step(alch_nb_ctx* ctx, const double* d_pos, const double* d_lambda,
                                    const alch_nb_out* out) {
  if (!ctx) return ALCH_NB_E_INVALID_ARG;
  if (!is_bound(ctx)) return ALCH_NB_E_NOT_BOUND;
  if (!d_pos || !d_lambda) return ALCH_NB_E_INVALID_ARG;
  if (!ctx->stream) return ALCH_NB_E_UNSUPPORTED;  // capture needs a non-null stream
  destroy_graph(ctx);
  HIPCHK(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
  alch_nb_status r = enqueue_compute(ctx, d_pos, d_lambda, ALCH_NB_AUTO_REBUILD, out, false);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(ctx->stream, &g);
  if (r != ALCH_NB_OK) {
    if (g) hipGraphDestroy(g);
    return r;
  }
  if (e != hipSuccess) return hip_fail(ctx, e);
  ctx->graph = g;
  HIPCHK(hipGraphInstantiate(&ctx->gexec, ctx->graph, nullptr, nullptr, 0));
  return ALCH_NB_OK;
}

alch_nb_status alch_nb_launch_step(alch_nb_ctx* ctx) {
  if (!ctx) return ALCH_NB_E_INVALID_ARG;
  if (!ctx->gexec) return ALCH_NB_E_NOT_BOUND;
  HIPCHK(hipGraphLaunch(ctx->gexec, ctx->stream));
  return ALCH_NB_OK;
}

int32_t alch_nb_last_hip_error(const alch_nb_ctx* ctx) { return ctx ? (int32_t)ctx->last_hip : 0; }

void alch_nb_destroy(alch_nb_ctx* ctx) {
  if (!ctx) return;
  if (ctx->bound && ctx->stream) hipStreamSynchronize(ctx->stream);
  if (ctx->static_dev >= 0) anb_static_release(ctx);
  destroy_graph(ctx);
  for (auto& e : ctx->ev) hipEventDestroy(e);
  delete ctx;
}

alch_nb_status alch_nb_backward(alch_nb_ctx* ctx, const double* d_pos, const double* d_lambda,
                                const double* d_grad_energy, const alch_nb_grad* grad) {
  if (!ctx) return ALCH_NB_E_INVALID_ARG;
  if (!is_bound(ctx)) return ALCH_NB_E_NOT_BOUND;
  if (!d_pos || !d_lambda || !d_grad_energy || !grad) return ALCH_NB_E_INVALID_ARG;
  (void)d_lambda;  // the lambda factors of the last forward are kept on the device
  const Dev& d = ctx->dev;
  if (grad->d_pos || grad->d_lambda)
    HIPCHK(launch_backward_finish(d, ctx->stream, ctx->p.precision, d_grad_energy, grad->d_pos, grad->d_lambda));
  if (grad->d_sigma || grad->d_sqrt_epsilon || grad->d_charge || grad->d_epsilon) {
    if (ctx->T > kMaxTypes || ctx->pme) return ALCH_NB_E_UNSUPPORTED;
    HIPCHK(launch_param_grads(d, ctx->stream, ctx->pc, ctx->p.precision, ctx->p.schedule, d_grad_energy,
                              grad->d_sigma, grad->d_sqrt_epsilon, grad->d_charge, grad->d_epsilon));
  }
  return ALCH_NB_OK;
}

alch_nb_status alch_nb_dihedrals(alch_nb_ctx* ctx, const double* d_pos, int32_t n_cv, const int32_t* d_idx,
                                 double* d_xi, double* d_dxi, const double* d_mass_inv, double* d_msum,
                                 const double* d_s, const double* d_kappa, double* d_u_dafed, double* d_forces) {
  if (!ctx) return ALCH_NB_E_INVALID_ARG;
  if (!is_bound(ctx)) return ALCH_NB_E_NOT_BOUND;
  if (n_cv < 0 || (n_cv > 0 && (!d_pos || !d_idx || !d_xi || !d_dxi))) return ALCH_NB_E_INVALID_ARG;
  if ((d_s == nullptr) != (d_kappa == nullptr)) return ALCH_NB_E_INVALID_ARG;
  if (n_cv == 0) return ALCH_NB_OK;
  HIPCHK(launch_dihedrals(ctx->stream, d_pos, n_cv, d_idx, d_xi, d_dxi, d_mass_inv, d_msum, d_s, d_kappa, d_u_dafed,
                          d_forces, ctx->dev.reps, ctx->dev.atom_rep, ctx->N, ctx->dev.flags));
  return ALCH_NB_OK;
}

int64_t alch_nb_opes_state_size(int32_t capacity) {
  if (capacity < 1) return -1;
  return (int64_t)OPES_HEADER + 2 * OPES_GRID_N + 2 * (int64_t)capacity;
}

alch_nb_status alch_nb_opes_init(alch_nb_ctx* ctx, double* d_state, int32_t capacity, double kT, double sigma,
                                 double barrier_std, double barrier_expl, double theta0) {
  if (!ctx || !d_state || capacity < 1 || !(kT > 0) || !(sigma > 0) || !(barrier_std > kT) ||
      !(barrier_expl > kT) || !std::isfinite(theta0))
    return ALCH_NB_E_INVALID_ARG;
  if (!is_bound(ctx)) return ALCH_NB_E_NOT_BOUND;
  HIPCHK(launch_opes_init(ctx->stream, d_state, capacity, kT, sigma, barrier_std, barrier_expl, theta0));
  return ALCH_NB_OK;
}

alch_nb_status alch_nb_opes_update(alch_nb_ctx* ctx, double* d_state, const double* d_dudl, double* d_lambda_out,
                                   int32_t deposit) {
  if (!ctx || !d_state) return ALCH_NB_E_INVALID_ARG;
  if (!is_bound(ctx)) return ALCH_NB_E_NOT_BOUND;
  HIPCHK(launch_opes(ctx->stream, d_state, d_dudl, d_lambda_out, deposit != 0));
  return ALCH_NB_OK;
}

// ------------------------------------------------------------------ lambda dynamics

static bool ld_params_ok(const alch_nb_ld_params* q) {
  if (!q) return false;
  if (q->capacity < 1 || q->ti_bins < 1 || q->n_cv < 0) return false;
  if (!(q->kT > 0) || !(q->mass > 0) || !(q->friction >= 0) || !(q->dt > 0) || !(q->sigma > 0)) return false;
  if (q->stride > 0 && (!(q->barrier_std > q->kT) || !(q->barrier_expl > q->kT))) return false;
  if (!(q->compress >= 0)) return false;
  if (q->n_cv > 0 && (!(q->kT_s > 0) || !(q->friction_s >= 0))) return false;
  return (long long)q->capacity * 6 + 2LL * q->ti_bins < (1LL << 40);
}

int64_t alch_nb_ld_state_size(const alch_nb_ld_params* q, int32_t n_replicas) {
  if (!ld_params_ok(q) || n_replicas < 1) return -1;
  return ld_state_words(n_replicas, q->n_cv, q->capacity, q->ti_bins);
}

alch_nb_status alch_nb_ld_layout(const alch_nb_ld_params* q, int32_t n_replicas, int64_t* o, int32_t n) {
  if (!ld_params_ok(q) || n_replicas < 1 || !o || n < 18) return ALCH_NB_E_INVALID_ARG;
  const long long rw = ld_rep_words(q->capacity, q->ti_bins);
  const long long cv = LD_HEADER + n_replicas * rw;
  const int64_t v[18] = {LD_HEADER, rw, LD_R_THETA, LD_R_P, LD_R_LAMBDA, LD_R_LAST_LAMBDA, LD_R_U, LD_R_DU,
                         LD_R_FTHETA, LD_R_N, LD_R_NSTD, LD_R_NEXPL, LD_REP_HEADER, LD_REP_HEADER + 3LL * q->capacity,
                         LD_REP_HEADER + 6LL * q->capacity, cv + LD_C_HEADER, cv + LD_C_HEADER + q->n_cv,
                         cv + LD_C_HEADER + 4LL * q->n_cv};
  for (int i = 0; i < 18; ++i) o[i] = v[i];
  return ALCH_NB_OK;
}

alch_nb_status alch_nb_ld_init(alch_nb_ctx* ctx, const alch_nb_ld_params* q, double* d_state, const double* d_theta0,
                               const double* d_s0, const double* d_mass_s, const double* d_kappa) {
  if (!ctx || !ld_params_ok(q) || !d_state || !d_theta0) return ALCH_NB_E_INVALID_ARG;
  if (q->n_cv > 0 && (!d_s0 || !d_mass_s || !d_kappa)) return ALCH_NB_E_INVALID_ARG;
  if (!is_bound(ctx)) return ALCH_NB_E_NOT_BOUND;
  LdInit in{};
  in.K = ctx->K;
  in.n_cv = q->n_cv;
  in.cap = q->capacity;
  in.bins = q->ti_bins;
  in.stride = q->stride;
  in.kT = q->kT;
  in.mass = q->mass;
  in.gamma = q->friction;
  in.dt = q->dt;
  in.sigma = q->sigma;
  in.compress = q->compress;
  in.kT_s = q->kT_s;
  in.gamma_s = q->friction_s;
  in.de_std = q->barrier_std;
  in.de_expl = q->barrier_expl;
  HIPCHK(launch_ld_init(ctx->stream, d_state, ld_state_words(ctx->K, q->n_cv, q->capacity, q->ti_bins), in, d_theta0,
                        d_s0, d_mass_s, d_kappa));
  ctx->ld_ncv = q->n_cv;
  return ALCH_NB_OK;
}

alch_nb_status alch_nb_ld_step(alch_nb_ctx* ctx, double* d_state, const double* d_dudl, const double* d_xi,
                               const double* d_noise, int32_t noise_rows, double* d_lambda_out) {
  if (!ctx || !d_state || !d_dudl || !d_noise || noise_rows < 1) return ALCH_NB_E_INVALID_ARG;
  if (!is_bound(ctx)) return ALCH_NB_E_NOT_BOUND;
  if (ctx->ld_ncv < 0) return ALCH_NB_E_NOT_BOUND;  // no state initialised
  if ((ctx->ld_ncv > 0) != (d_xi != nullptr)) return ALCH_NB_E_INVALID_ARG;
  HIPCHK(launch_ld_step(ctx->stream, d_state, ctx->K, ctx->ld_ncv, d_dudl, d_xi, d_noise, noise_rows, d_lambda_out,
                        ctx->dev.flags, LdCv{}));
  return ALCH_NB_OK;
}

alch_nb_status alch_nb_ld_step_dafed(alch_nb_ctx* ctx, double* d_state, const double* d_dudl, const double* d_pos,
                                     const int32_t* d_idx, double* d_xi, double* d_u_dafed, double* d_forces,
                                     const double* d_noise, int32_t noise_rows, double* d_lambda_out) {
  if (!ctx || !d_state || !d_dudl || !d_pos || !d_idx || !d_noise || noise_rows < 1) return ALCH_NB_E_INVALID_ARG;
  if (!is_bound(ctx)) return ALCH_NB_E_NOT_BOUND;
  if (ctx->ld_ncv < 0) return ALCH_NB_E_NOT_BOUND;  // no state initialised
  if (ctx->ld_ncv == 0) return ALCH_NB_E_INVALID_ARG;  // no auxiliary variables to couple
  const LdCv cv{d_pos, d_idx, d_xi, d_u_dafed, d_forces, ctx->dev.reps, ctx->dev.atom_rep, ctx->N};
  HIPCHK(launch_ld_step(ctx->stream, d_state, ctx->K, ctx->ld_ncv, d_dudl, nullptr, d_noise, noise_rows,
                        d_lambda_out, ctx->dev.flags, cv));
  return ALCH_NB_OK;
}

alch_nb_status alch_nb_ld_free_energy(alch_nb_ctx* ctx, const double* d_state, double* d_out) {
  if (!ctx || !d_state || !d_out) return ALCH_NB_E_INVALID_ARG;
  if (!is_bound(ctx)) return ALCH_NB_E_NOT_BOUND;
  HIPCHK(launch_ld_free_energy(ctx->stream, d_state, ctx->K, d_out));
  return ALCH_NB_OK;
}

// ------------------------------------------------------------------ replica exchange

alch_nb_status alch_nb_hrex_init(alch_nb_ctx* ctx, int32_t* d_state_of, int64_t* d_stats) {
  if (!ctx || !d_state_of || !d_stats) return ALCH_NB_E_INVALID_ARG;
  if (!is_bound(ctx)) return ALCH_NB_E_NOT_BOUND;
  if (ctx->K < 2 || ctx->K > kHrexMax) return ALCH_NB_E_UNSUPPORTED;
  HIPCHK(launch_hrex_init(ctx->stream, d_state_of, reinterpret_cast<long long*>(d_stats), ctx->K));
  return ALCH_NB_OK;
}

alch_nb_status alch_nb_hrex_exchange(alch_nb_ctx* ctx, const double* d_terms, const double* d_lambda_states,
                                     int32_t* d_state_of, double* d_lambda, const double* d_uniform, int32_t rows,
                                     double kT, int64_t* d_stats) {
  if (!ctx || !d_terms || !d_lambda_states || !d_state_of || !d_lambda || !d_uniform || rows < 1 || !(kT > 0) ||
      !d_stats)
    return ALCH_NB_E_INVALID_ARG;
  if (!is_bound(ctx)) return ALCH_NB_E_NOT_BOUND;
  if (ctx->p.schedule != ALCH_NB_LBF_DSF || ctx->K < 2 || ctx->K > kHrexMax) return ALCH_NB_E_UNSUPPORTED;
  HIPCHK(launch_hrex(ctx->stream, d_terms, d_lambda_states, d_state_of, d_lambda, d_uniform, rows, kT,
                     reinterpret_cast<long long*>(d_stats), ctx->K));
  return ALCH_NB_OK;
}

alch_nb_status alch_nb_capture_begin(alch_nb_ctx* ctx) {
  if (!ctx) return ALCH_NB_E_INVALID_ARG;
  if (!is_bound(ctx)) return ALCH_NB_E_NOT_BOUND;
  if (!ctx->stream) return ALCH_NB_E_UNSUPPORTED;
  destroy_graph(ctx);
  HIPCHK(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
  ctx->capturing = true;
  return ALCH_NB_OK;
}

alch_nb_status alch_nb_capture_end(alch_nb_ctx* ctx) {
  if (!ctx) return ALCH_NB_E_INVALID_ARG;
  if (!ctx->stream) return ALCH_NB_E_UNSUPPORTED;
  hipGraph_t g = nullptr;
  ctx->capturing = false;
  HIPCHK(hipStreamEndCapture(ctx->stream, &g));
  ctx->graph = g;
  HIPCHK(hipGraphInstantiate(&ctx->gexec, ctx->graph, nullptr, nullptr, 0));
  return ALCH_NB_OK;
}

// ------------------------------------------------------------------ autotuner

// Cache key: precision, schedule, log2 size bucket, boxes, density bucket
// (atoms per nm^3) and cutoff (0.01 A).
static std::string tune_key(const alch_nb_ctx* ctx) {
  double vol = 0;
  for (const auto& r : ctx->reps) vol += r.box[0] * r.box[1] * r.box[2];
  const double rho = vol > 0 ? 1000.0 * ctx->N / vol : 0.0;
  char buf[160];
  std::snprintf(buf, sizeof(buf), "gfx950|p%d|s%d|n%d|k%d|rho%d|rc%d", ctx->p.precision, ctx->p.schedule,
                (int)std::lround(std::log2(std::max(1, ctx->N))), ctx->K, (int)std::lround(rho / 10.0) * 10,
                (int)std::lround(100.0 * ctx->p.cutoff));
  return buf;
}

static int tune_cache_lookup(const std::string& key) {
  const char* path = std::getenv("ALCHNB_TUNE_CACHE");
  if (!path) return -1;
  std::ifstream f(path);
  if (!f) return -1;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string txt = ss.str();
  const std::string pat = "\"" + key + "\":";
  const size_t at = txt.find(pat);
  if (at == std::string::npos) return -1;
  const int v = std::atoi(txt.c_str() + at + pat.size());
  return (v >= 0 && v < kNumVariants) ? v : -1;
}

static void tune_cache_store(const std::string& key, int variant) {
  const char* path = std::getenv("ALCHNB_TUNE_CACHE");
  if (!path) return;
  std::string txt;
  {
    std::ifstream f(path);
    if (f) {
      std::stringstream ss;
      ss << f.rdbuf();
      txt = ss.str();
    }
  }
  // entries are one per line: "key": variant
  std::string out = "{\n";
  std::istringstream in(txt);
  std::string line;
  bool first = true;
  const std::string pat = "\"" + key + "\":";
  while (std::getline(in, line)) {
    const size_t q = line.find('"');
    if (q == std::string::npos || line.find(pat) != std::string::npos) continue;
    std::string ent = line.substr(q);
    while (!ent.empty() && (ent.back() == ',' || ent.back() == ' ')) ent.pop_back();
    out += (first ? "  " : ",\n  ") + ent;
    first = false;
  }
  out += (first ? "  " : ",\n  ") + pat + " " + std::to_string(variant) + "\n}\n";
  std::ofstream f(path, std::ios::trunc);
  f << out;
}

alch_nb_status alch_nb_autotune(alch_nb_ctx* ctx, const double* d_pos, const double* d_lambda, int32_t reps) {
  if (!ctx) return ALCH_NB_E_INVALID_ARG;
  if (!is_bound(ctx)) return ALCH_NB_E_NOT_BOUND;
  if (!d_pos || !d_lambda || reps < 1) return ALCH_NB_E_INVALID_ARG;
  alch_nb_status r = enqueue_compute(ctx, d_pos, d_lambda, ALCH_NB_AUTO_REBUILD, nullptr, false);
  if (r != ALCH_NB_OK) return r;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  int best = ctx->variant;
  float best_ms = 1e30f;
  for (int v = 0; v < kNumVariants; ++v) {
    r = alch_nb_set_variant(ctx, v);
    if (r != ALCH_NB_OK) break;
    const TileShape sh = shape_of(ctx);
    HIPCHK(launch_tile(ctx->dev, ctx->stream, ctx->pc, ctx->p.precision, ctx->p.schedule, sh, d_pos));  // warm-up
    HIPCHK(hipEventRecord(e0, ctx->stream));
    for (int k = 0; k < reps; ++k)
      HIPCHK(launch_tile(ctx->dev, ctx->stream, ctx->pc, ctx->p.precision, ctx->p.schedule, sh, d_pos));
    HIPCHK(hipEventRecord(e1, ctx->stream));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    if (ms < best_ms) {
      best_ms = ms;
      best = v;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (r != ALCH_NB_OK) return r;
  r = alch_nb_set_variant(ctx, best);
  if (r != ALCH_NB_OK) return r;
  // restore the force accumulators and outputs of a regular evaluation
  r = enqueue_compute(ctx, d_pos, d_lambda, 0, nullptr, false);
  if (r != ALCH_NB_OK) return r;
  HIPCHK(hipStreamSynchronize(ctx->stream));
  ctx->tuned_ms = best_ms / reps;
  tune_cache_store(tune_key(ctx), best);
  return ALCH_NB_OK;
}

}  // extern "C"
