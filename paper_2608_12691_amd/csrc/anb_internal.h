// Internal layout shared by the host side and the HIP kernels of libalchnb.
//
// Spatial organisation (per box, per group: the solute atoms and the
// environment atoms of a box each get their own column grid so that no
// cluster mixes the two groups):
//   column  - an x-y cell of the group's grid spanning the whole box in z;
//   super-cluster (SC) - 64 consecutive z-sorted atoms of one column, split
//             2 x 2 x 2 into 8 clusters (fewer if the column runs out);
//   cluster - 8 atom slots; empty slots are padding.
// A list entry pairs one i-SC with one j-cluster and one periodic image
// shift; an 8-bit mask says which of the SC's clusters interact with it and
// eight 64-bit masks give the atom pairs (padding, exclusions, i<j inside a
// cluster).  A work unit is a run of consecutive entries of one i-SC.
#pragma once
#include <stdint.h>

namespace anb {

constexpr int kCl = 8;           // atom slots per cluster
constexpr int kScCl = 8;         // clusters per super-cluster
constexpr int kSc = 64;          // atom slots per super-cluster
// grid barrier of the fused list build: word 0 top arrival count, word 1
// generation, word kBarStride*(g+1) arrival count of block group g
constexpr int kBarGroups = 8;
constexpr int kBarStride = 16;  // counters on separate 64-byte lines
constexpr int kBarWords = kBarStride * (kBarGroups + 1);
// the tile kernel's launch has at most kMaxWaves waves
constexpr int kMaxWaves = 8192;
constexpr int kRedChunks = 16;   // unit chunks per box in the final reduction
constexpr int kAlchTileCost = 12;  // cost of a solute-solvent tile, in plain tiles (measured: 12-16 best)
constexpr uint32_t kUnitStart = 1u << 31;  // ent_info bit: a work unit starts at this entry
constexpr int kStrips = 8;       // search waves per super-cluster (neighbour columns dealt round-robin)
constexpr double kKe = 332.06371;
constexpr int kNTerms = 10;  // energy-term slots per box

// per-unit energy accumulators (FP64)
enum { ACC_SOLV = 0, ACC_SOLU = 1, ACC_A0 = 2, ACC_A1 = 3, ACC_A2 = 4, ACC_NPAIR = 5, NACC = 6 };
// entry kinds
enum { KIND_SOLV = 0, KIND_SOLU = 1, KIND_ALCH = 2 };

// Unit header int4: (super-cluster, first entry, end entry, replica | flag);
// the flag marks the units of solute super-clusters, which hold every
// solute-solute and solute-solvent entry (solute super-clusters come first
// in each replica and the half list pairs a super-cluster only with
// clusters of itself and later ones).
constexpr int kUnitSolute = 1 << 30;
__host__ __device__ inline int unit_rep(int w) { return w & (kUnitSolute - 1); }

struct GridInfo {
  int replica, is_solute;
  int atom_off, n_atoms;   // range in grid_atoms[]
  int col_base, ncx, ncy;  // columns [col_base, col_base + ncx*ncy)
  int sc_base, sc_cap;     // super-cluster slots [sc_base, sc_base + sc_cap)
  int pad_;
  double wx, wy;           // column widths
};

struct ReplicaInfo {
  double box[3];
  int atom_off, n_atoms;
  int grid0, n_grids;
  int sc_begin, sc_end;    // SC slot range of the replica
};

// Per-replica lambda factors, recomputed on the device every call.
//   Beutler: a[0] = lv, a[1] = le, a[2] = dlv/dlambda, a[3] = dle/dlambda
//   LBF:     a[0] = hA, a[1] = hB, a[2] = dhA, a[3] = dhB
struct LamState {
  double a[4];
  float f[4];
};

// Entry info word: bits 0-7 i-cluster mask, 8-9 kind, 16-20 shift code
// (sx+1) + 3 (sy+1) + 9 (sz+1).
__host__ __device__ inline uint32_t ent_pack(uint32_t imask, uint32_t kind, uint32_t shift) {
  return imask | (kind << 8) | (shift << 16);
}

// Smooth particle-mesh Ewald (electrostatics ALCH_NB_ELEC_PME).  Per box
// one complex FP64 grid, z fastest, holding the solute charge grid in the
// real part and the solvent grid in the imaginary part (after the forward
// transform their spectra mixed; after the convolution and the inverse
// transform the two potential grids G_S, G_W), and two int64 fixed-point
// spreading grids (S, W) that the first FFT pass reads and clears.  Per box
// and axis an FFT root table exp(-2 pi i k/n) and the B-spline moduli
// |b(m)|^2.  Partial sums per box: kPmeParts blocks of the convolution and
// of the excluded-pair pass each write their own PME_NPART slots; the
// self energies and group charges are constants of the binding.  The charge
// grids count pme_qscale units per e, a power of two with
// pme_qscale * max_box sum |q_i| <= 2^62 (a grid value never exceeds the
// box's sum of |q_i|: the spline weights of an atom are at most 1), at most
// 2^52.
constexpr int kPmeMaxN = 512;       // grid points per edge at most
constexpr int kPmeMinOrder = 4, kPmeMaxOrder = 6;
constexpr int kPmeParts = 256;  // partial-sum slots per box (one per thread of the final reduction's block)
enum {
  PME_E_SS = 0, PME_E_WW = 1, PME_E_SW = 2,   // reciprocal parts (convolution)
  PME_C_SS = 3, PME_C_WW = 4, PME_C_SW = 5,   // excluded-pair parts
  PME_NPART = 6
};
// per-box constants: self energies of the two groups and their charges
enum { PME_K_SELF_S = 0, PME_K_SELF_W = 1, PME_K_Q_S = 2, PME_K_Q_W = 3 };
struct PmeBox {
  int n[3];          // grid points per axis
  int tab[3];        // offsets of the axis tables in pme_roots and pme_bmod
  int tiles[3];      // first FFT tile of this box in the pass along each axis (prefix over boxes)
  int pair0, npair;  // its excluded pairs in pme_pairs
  int pad_;
  long long off;     // first grid point of the box
  double L[3];       // box edges
};
// an excluded pair of one box: global atom indices, k_e q_i q_j, and the
// part it belongs to (0 solute-solute, 1 solvent-solvent, 2 solute-solvent)
struct PmePair {
  int i, j;
  double qq;
  int kind, pad_;
};
// x-lines of a box that come before their mirror line (-iy, -iz) or are
// their own mirror, and how many of them (each with its mirror) a tile of
// the fused x pass holds (about 256 points a side: tiles of a few hundred
// points give these latency-bound passes more blocks; measured on a 45^3
// grid, 4-5 lines beat 2 and 8-16)
__host__ __device__ inline int canon_lines(int n1, int n2) {
  return ((n1 - 1) / 2) * n2 + (n2 / 2 + 1) * (n1 % 2 == 0 ? 2 : 1);
}
__host__ __device__ inline int pair_tile_lines(int n0) {
  const int t = 256 / n0;
  return t < 1 ? 1 : (t > 8 ? 8 : t);
}
// lines of an FFT tile along an axis of n points (about 256 points)
__host__ __device__ inline int tile_lines(int n) {
  const int t = 256 / n;
  return t < 1 ? 1 : (t > 16 ? 16 : t);
}

// Device view of the workspace.
struct Dev {
  int n_atoms, n_reps, n_grids, n_cols, sc_cap, ent_cap, unit_cap, n_types;
  // static tables
  const int* atom_type;      // [N]
  const int* atom_grid;      // [N]
  const int* atom_rep;       // [N] box of each atom
  const int* atom_comp;      // [N] connected component of the exclusion graph (global id)
  const double4* sc_box;     // [SC] box lengths of the SC's replica (SC ranges are fixed per grid)
  const int* grid_atoms;     // [N] atoms of each grid, concatenated
  const GridInfo* grids;     // [G]
  const ReplicaInfo* reps;   // [K]
  const int* excl_start;     // [N+1]
  const int* excl_j;         // [M] global, sorted per row
  const double* type_sigma;  // [T]
  const double* type_eps;    // [T]
  const double* type_q;      // [T]
  int* col_grid;             // [C] grid of each column
  // list state
  double* x_build;           // [N*3]
  double* xw;                // [N*3] wrapped positions at build
  int* atom_col;             // [N]
  int* col_count;            // [C]
  int* col_start;            // [C]
  int* col_fill;             // [C]
  int* col_sc;               // [C] first SC of the column
  int* col_nsc;              // [C]
  double* bucket_z;          // [N] wrapped z of the bucket's atom (sort keys)
  int* bucket;               // [N]
  int* sorted;               // [N]
  int* sc_first;             // [SC] offset into sorted
  int* sc_n;                 // [SC] atoms
  int* sc_col;               // [SC]
  double* sc_origin;         // [SC*3]
  double* sc_bbox;           // [SC*6] lo xyz, hi xyz
  double* cl_bbox;           // [SC*8*6]
  int* cl_n;                 // [SC*8]
  int* slot_atom;            // [SC*64] atom index or -1
  int* atom_slot;            // [N]
  double4* atom_off;         // [N] build-time offset of the atom from its SC origin, .w = slot + 1 (set with the slots)
  double4* atom_box;         // [N] box of the atom's replica (set with the slots)
  double4* slot_xw;          // [SC*64] build-time wrapped position of the slot's atom
  int* slot_comp;            // [SC*64] exclusion component of the slot's atom (-1 = padding)
  int* slot_type;            // [SC*64] atom type of the slot (0 for padding)
  float2* se32;              // [SC*64] sigma/2, 2 sqrt(eps)
  double2* se64;             // [SC*64]
  float* q32;                // [SC*64] q sqrt(k_e)
  double* q64;               // [SC*64]
  int* sc_ecount;            // [SC]
  int* sc_estart;            // [SC]
  int* strip_count;          // [SC*kStrips] entries found by each search wave
  int* strip_start;          // [SC*kStrips]
  int* sc_ustart;            // [SC]
  int* ent_jc;               // [E]
  uint32_t* ent_info;        // [E]
  double4* ent_off;          // [E] offset of the entry's j-cluster image from its i-SC origin (FP64, set with the masks)
  int* ent_isc;              // [E]
  unsigned long long* ent_mask;  // [E*8]
  int4* units;               // [U] sc, e0, e1, replica
  // start record of each wave of the tile launch (written with the units
  // for the launch's wave count, ctr[CTR_WAVES]): run start, run length,
  // 1 if the run holds solute units; the run's first unit and its entries
  int4* wrec;                // [kMaxWaves]
  int4* wrec_u0;             // [kMaxWaves]
  int* wrec_jc;              // [kMaxWaves*8]
  uint32_t* wrec_info;       // [kMaxWaves*8]
  double4* wrec_off;         // [kMaxWaves*8]
  int* rep_ustart;           // [K+1]
  int* ctr;                  // [16] counters, see CTR_*
  unsigned int* flags;       // [1] sticky flags
  int* rebuild;              // [1]
  unsigned int* barrier;     // [kBarWords] grid barrier: top count, generation, group counts
  // per call
  float4* pos32;             // [SC*64] local x, y, z, q
  double4* pos64;            // [SC*64]
  unsigned long long* ffix;  // [3*SC*64] fixed-point forces, component-major
  double* unit_acc;          // [NACC][U] per-unit partial sums (component-major)
  double* chunk_acc;         // [K][kRedChunks][NACC] partial sums of unit chunks
  unsigned int* red_done;    // [K] chunks reduced (the last one finishes its box; reset to 0)
  LamState* lam;             // [K]
  double* last_dudl;         // [K] dU/dlambda of the last forward
  unsigned long long* pg_fix;  // [3][SC*64] parameter-gradient sums per slot (fixed point), cleared after each pass
  const float4* tp32;        // [T*T] type-pair sigma, 4 eps, k_e q q, 1/sigma^6 (rounded from FP64)
  const float4* dsf32;       // [kDsfEntries] FP32 pieces of r D(r), then r (-r dD/dr), per interval
  const double4* tp64;       // [T*T]
  const double* pot64;       // [kPot64Words] FP64 potential constants of the solute units (see pot64_words)
  // PME (pme_box == nullptr: DSF electrostatics)
  const PmeBox* pme_box;     // [K]
  double2* pme_grid;         // [pme_points]
  unsigned long long* pme_q; // [2][pme_points] charge spreading grids S, W (fixed point)
  const double2* pme_roots;  // per box and axis: exp(-2 pi i k/n), k < n
  const double* pme_bmod;    // per box and axis: |b(m)|^2
  double* pme_part;          // [K][kPmeParts][PME_NPART]
  double* pme_infl;          // [pme_points] influence function C(m) (written once at bind)
  double* pme_const;         // [K][4] self energies and group charges (written once at bind)
  const PmePair* pme_pairs;  // excluded pairs of all boxes
  long long pme_points;      // grid points of all boxes
  int pme_tiles[3];          // FFT tiles of all boxes per axis
  int pme_order;
  double pme_alpha;          // Ewald splitting parameter
  double pme_qscale;         // fixed-point units per e of the charge grids
};

// Replica exchange: boxes per context it handles, and the terms per box.
constexpr int kHrexMax = 4096;
constexpr int NTERMS_DEV = 10;

// Lambda-dynamics state (doubles): a header, one record per replica (theta
// and its OPES kernels and TI bins), then the auxiliary-variable section.
enum {
  LD_K = 0, LD_NCV = 1, LD_CAP = 2, LD_BINS = 3, LD_STRIDE = 4, LD_KT = 5, LD_MASS = 6, LD_GAMMA = 7, LD_DT = 8,
  LD_SIGMA = 9, LD_COMPRESS = 10, LD_KT_S = 11, LD_GAMMA_S = 12, LD_DE_STD = 13, LD_DE_EXPL = 14, LD_HEADER = 16
};
// per replica: header, then Standard kernels (centres, weights, widths:
// cap each), Explore kernels (same), TI sums and counts (bins each)
enum {
  LD_R_THETA = 0, LD_R_P = 1, LD_R_LAMBDA = 2, LD_R_LAST_LAMBDA = 3, LD_R_DLAM = 4, LD_R_U = 5, LD_R_DU = 6,
  LD_R_FTHETA = 7, LD_R_N = 8, LD_R_NSTD = 9, LD_R_NEXPL = 10, LD_R_RBAR_STD = 11, LD_R_RBAR_EXPL = 12,
  LD_REP_HEADER = 16
};
// auxiliary section: step count, then s, p, mass, kappa, last force (n_cv each)
enum { LD_C_N = 0, LD_C_HEADER = 8 };
__host__ __device__ inline long long ld_rep_words(int cap, int bins) {
  return LD_REP_HEADER + 6LL * cap + 2LL * bins;
}
__host__ __device__ inline long long ld_state_words(int K, int n_cv, int cap, int bins) {
  return LD_HEADER + (long long)K * ld_rep_words(cap, bins) + LD_C_HEADER + 5LL * n_cv;
}
struct LdInit {
  int K, n_cv, cap, bins, stride;
  double kT, mass, gamma, dt, sigma, compress, kT_s, gamma_s, de_std, de_expl;
};

enum { CTR_NSC = 0, CTR_NENT = 1, CTR_NUNIT = 2, CTR_NBUILD = 3, CTR_ENT_NEED = 4, CTR_UNIT_NEED = 5, CTR_TILES = 6,
       CTR_WAVES = 7 };

constexpr int kMaxTypes = 256;  // atom types supported by the parameter-gradient pass

// lambda/OPES state layout (doubles): header, bias and derivative on the
// output grid, kernel centres and Standard weights
enum {
  OPES_THETA = 0, OPES_LAMBDA = 1, OPES_DLAM = 2, OPES_U = 3, OPES_DU = 4, OPES_FTHETA = 5, OPES_KT = 6,
  OPES_SIGMA = 7, OPES_DE_STD = 8, OPES_DE_EXPL = 9, OPES_N = 10, OPES_CAP = 11, OPES_S_STD = 12,
  OPES_S_EXPL = 13, OPES_W_STD = 14, OPES_HEADER = 16, OPES_GRID_N = 101
};

}  // namespace anb
