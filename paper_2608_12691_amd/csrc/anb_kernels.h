// Launchers of the HIP kernels (host side of libalchnb).
#pragma once
#include <hip/hip_runtime.h>

#include "alch_nb.h"
#include "anb_internal.h"

namespace anb {

// Pair-potential constants, precomputed on the host in FP64.
constexpr int kPot64Words = 12;

struct PotConsts {
  double rc, rc2, rs, inv_w;   // cutoff, its square, switch start, 1/width (0 = no switch)
  double alpha, A, B, c2a;     // DSF: a, erfc(a rc)/rc, slope, 2a/sqrt(pi)
  double sc_alpha;             // Beutler soft-core alpha
  double inv_h;                // intervals per unit of r in the FP32 DSF table (a power of two)
};

// The FP32 path reads r D(r) and r (-r dD/dr) (D the electrostatic pair
// function, shift included) from cubic Hermite pieces on kDsfN + 1 equal
// intervals of width 1/inv_h starting at r = 0, with rc * inv_h <= kDsfN;
// each interval holds two float4 of coefficients in the local variable t
// in [0, 1].
constexpr int kDsfN = 256;
constexpr int kDsfEntries = 2 * (kDsfN + 1);

constexpr int kMaxEpu = 8;  // entries per work unit at most (LDS staging of j-forces)

struct TileShape {
  int epu;      // entries per work unit at most
  int tiles;    // 64-pair tiles per work unit at most (past its first entry)
  int blocks;   // blocks of 256 threads (4 waves); waves take equal runs of units
};

// fused_blocks > 0: one launch of the fused build with that many blocks
// (all resident at once); 0: one launch per phase.
hipError_t launch_list_build(const Dev& d, hipStream_t st, const double* pos, double r_list, const TileShape& shape,
                             int fused_blocks);
// Resident blocks per compute unit of the fused list kernel (0 on error).
int list_fused_max_blocks();
// work units and their partition over the waves of a tile launch of this shape
hipError_t launch_units(const Dev& d, hipStream_t st, const TileShape& shape);  // work units of this shape
hipError_t launch_export(const Dev& d, hipStream_t st, double r_list, int* out, long long cap,
                         unsigned long long* counter);
hipError_t launch_init(const Dev& d, hipStream_t st);
hipError_t launch_prepare(const Dev& d, hipStream_t st, const double* pos, const double* lambda, int mode,
                          double half_skin, int schedule);
// The FP64 constants the tile kernel's solute units read from the workspace
// (kPot64Words doubles, uploaded at bind).
void pot64_words(const PotConsts& pc, double* out);
hipError_t launch_tile(const Dev& d, hipStream_t st, const PotConsts& pc, int precision, int schedule,
                       const TileShape& shape, const double* xin);
hipError_t launch_finalize(const Dev& d, hipStream_t st, int precision, int schedule, double* terms,
                           double* forces, double* dudl, long long* n_pairs);
// Smooth-PME reciprocal space, self and excluded-pair parts of every box
// (after the tile kernel, before the final reduction that adds them).
// yz_planes > 0: the y and z transforms of each grid plane in one block
// (every box's y-z plane holds at most kPmePlanePts points; yz_planes is
// the largest x edge); 0: the y and z passes by line tiles.
constexpr int kPmePlanePts = 4096;
hipError_t launch_pme(const Dev& d, hipStream_t st, const double* pos, int schedule, int precision, int yz_planes);
// The influence-function table and the per-box constants (at bind).
hipError_t launch_pme_init(const Dev& d, hipStream_t st);
// pair inputs from the last forward's slot coordinates and list
hipError_t launch_param_grads(const Dev& d, hipStream_t st, const PotConsts& pc, int precision, int schedule,
                              const double* g_energy, double* d_sigma, double* d_sqrt_eps, double* d_charge, double* d_eps);
hipError_t launch_backward_finish(const Dev& d, hipStream_t st, int precision, const double* g_energy,
                                  double* d_pos, double* d_lambda);
hipError_t launch_dihedrals(hipStream_t st, const double* pos, int n_cv, const int* idx, double* xi, double* dxi,
                            const double* mass_inv, double* msum, const double* s, const double* kappa,
                            double* u_dafed, double* forces, const ReplicaInfo* reps, const int* atom_rep,
                            int n_atoms, unsigned int* flags);
hipError_t launch_opes_init(hipStream_t st, double* state, int cap, double kT, double sigma, double de_std,
                            double de_expl, double theta0);
hipError_t launch_opes(hipStream_t st, double* state, const double* dudl, double* lambda_out, int deposit);

// Fixed-point scale of the force accumulators (units per kcal/mol/A).
inline double fixed_scale(int precision) { return precision == 0 ? 4294967296.0 : 1099511627776.0; }

hipError_t launch_ld_init(hipStream_t st, double* state, long long words, const LdInit& in, const double* theta0,
                          const double* s0, const double* mass_s, const double* kappa);
// The d-AFED CVs evaluated inside the lambda-dynamics step (pos null: the
// step reads xi from its argument instead).
struct LdCv {
  const double* pos;
  const int* idx;
  double* xi_out;
  double* u_dafed;
  double* forces;
  const ReplicaInfo* reps;
  const int* atom_rep;
  int n_atoms;
};
hipError_t launch_ld_step(hipStream_t st, double* state, int K, int n_cv, const double* dudl, const double* xi,
                          const double* noise, int noise_rows, double* lam_out, unsigned int* flags,
                          const LdCv& cv);
hipError_t launch_hrex_init(hipStream_t st, int* state_of, long long* stats, int K);
hipError_t launch_hrex(hipStream_t st, const double* terms, const double* lam_states, int* state_of, double* lam_out,
                       const double* uniform, int rows, double kT, long long* stats, int K);
hipError_t launch_ld_free_energy(hipStream_t st, const double* state, int K, double* out);

}  // namespace anb

// Binding (alch_nb.cpp) and the library-owned device scratch (noalloc.hip).
alch_nb_status anb_bind(alch_nb_ctx* ctx, void* d_ws, size_t bytes, void* stream, int static_device);
bool anb_static_owns(const alch_nb_ctx* ctx, int device);
void anb_static_release(const alch_nb_ctx* ctx);
