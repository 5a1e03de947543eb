// Replica exchange between lambda states from the LBF basis energies (FP64).
//
// With the LBF potential (eq. 4) linear in its bases, the energy change of
// box a moved from state l to l' is (hA(l') - hA(l)) U_A,a + (hB(l') - hB(l))
// U_B,a, so one evaluation per box gives every neighbour swap's
// D = [U_a(l_s+1) - U_a(l_s) + U_b(l_s) - U_b(l_s+1)] / kT; a swap is
// accepted when D <= 0 or u < exp(-D).  Attempt n pairs the states (s, s+1)
// with s of parity n mod 2 (disjoint pairs, decided in parallel) and takes
// pair s's uniform deviate from row n mod rows of the caller's array.  The
// boxes' lambdas are rewritten in place, so an evaluation followed by this
// launch is one HREX step that a graph can replay.
#include <hip/hip_runtime.h>

#include "anb_internal.h"
#include "anb_kernels.h"
#include "pair_math.h"

namespace anb {

constexpr int kHrexBlk = 256;

__global__ void __launch_bounds__(kHrexBlk) k_hrex(const double* __restrict__ terms,
                                                   const double* __restrict__ lam_states, int* __restrict__ state_of,
                                                   double* __restrict__ lam_out, const double* __restrict__ uniform,
                                                   int rows, double kT, long long* __restrict__ stats, int K) {
  __shared__ int box_of[kHrexMax];
  const long long n = stats[0];
  for (int r = threadIdx.x; r < K; r += kHrexBlk) box_of[state_of[r]] = r;
  __syncthreads();
  const double* u = uniform + (size_t)(n % rows) * (K - 1);
  for (int s = (int)(n & 1) + 2 * threadIdx.x; s < K - 1; s += 2 * kHrexBlk) {
    const int a = box_of[s], b = box_of[s + 1];
    double ha0, hb0, ha1, hb1, d0, d1;
    lbf_switch(lam_states[s], ha0, hb0, d0, d1);
    lbf_switch(lam_states[s + 1], ha1, hb1, d0, d1);
    const double ua_a = terms[a * NTERMS_DEV + 4], ub_a = terms[a * NTERMS_DEV + 5];
    const double ua_b = terms[b * NTERMS_DEV + 4], ub_b = terms[b * NTERMS_DEV + 5];
    const double D = ((ha1 - ha0) * (ua_a - ua_b) + (hb1 - hb0) * (ub_a - ub_b)) / kT;
    const bool ok = D <= 0.0 || u[s] < exp(-D);
    stats[1 + s] += 1;
    if (ok) {
      stats[K + s] += 1;
      state_of[a] = s + 1;
      state_of[b] = s;
    }
  }
  __syncthreads();
  for (int r = threadIdx.x; r < K; r += kHrexBlk) lam_out[r] = lam_states[state_of[r]];
  if (threadIdx.x == 0) stats[0] = n + 1;
}

__global__ void __launch_bounds__(kHrexBlk) k_hrex_init(int* __restrict__ state_of, long long* __restrict__ stats,
                                                        int K) {
  for (int r = threadIdx.x; r < K; r += kHrexBlk) state_of[r] = r;
  for (int i = threadIdx.x; i < 2 * K - 1; i += kHrexBlk) stats[i] = 0;
}

hipError_t launch_hrex_init(hipStream_t st, int* state_of, long long* stats, int K) {
  hipLaunchKernelGGL(k_hrex_init, dim3(1), dim3(kHrexBlk), 0, st, state_of, stats, K);
  return hipGetLastError();
}

hipError_t launch_hrex(hipStream_t st, const double* terms, const double* lam_states, int* state_of, double* lam_out,
                       const double* uniform, int rows, double kT, long long* stats, int K) {
  hipLaunchKernelGGL(k_hrex, dim3(1), dim3(kHrexBlk), 0, st, terms, lam_states, state_of, lam_out, uniform, rows, kT,
                     stats, K);
  return hipGetLastError();
}

}  // namespace anb
