// Neighbour-list construction on the device.
//
// Each phase is a __device__ function written for 256-thread blocks: scans
// run in block 0, per-column sorts are block-wide, per-super-cluster and
// per-entry work is wave-wide.  The phases run either as separate kernels
// or, fused, as one cooperative kernel with grid barriers between them.
// Every phase is gated by the device flag *rebuild so that a captured step
// can always launch it: with the flag at 0 nothing is done.
//
// Placement is deterministic: atoms are ordered by (z, atom index) inside a
// column by a rank sort, super-clusters are split by ranks, and list
// entries are written at offsets from an exclusive scan of per-SC counts in
// a fixed candidate order.  No output position depends on atomic ordering.
#include <hip/hip_runtime.h>

#include "anb_internal.h"
#include "anb_kernels.h"

namespace anb {

constexpr int kBlk = 512;          // threads per block of every list kernel
constexpr int kWpb = kBlk / 64;     // waves per block

__device__ inline bool rebuild_on(const Dev& d) { return __atomic_load_n(d.rebuild, __ATOMIC_RELAXED) != 0; }

// canonical wrap x - L floor(x / L), without contraction
__device__ inline double wrap_canon(double x, double L) { return __dsub_rn(x, __dmul_rn(L, floor(x / L))); }

__device__ inline int gtid() { return blockIdx.x * blockDim.x + threadIdx.x; }
__device__ inline int gthreads() { return gridDim.x * blockDim.x; }
__device__ inline int gwave() { return blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }
__device__ inline int gwaves() { return gridDim.x * (blockDim.x >> 6); }

// ------------------------------------------------------------ block scans

// Exclusive scan of one int per thread over the block; *total = block sum.
__device__ int block_exclusive_scan(int v, int* total) {
  __shared__ int buf[kBlk];
  const int t = threadIdx.x, nt = blockDim.x;
  buf[t] = v;
  __syncthreads();
  for (int off = 1; off < nt; off <<= 1) {
    const int add = t >= off ? buf[t - off] : 0;
    __syncthreads();
    buf[t] += add;
    __syncthreads();
  }
  const int incl = buf[t];
  *total = buf[nt - 1];
  __syncthreads();
  return incl - v;
}

// Exclusive scan of src[0..n) into dst by one block; returns the total.
// src and dst may alias (values are read before they are overwritten).
__device__ int block_scan_array(const int* src, int* dst, int n) {
  const int per = (n + blockDim.x - 1) / blockDim.x;
  const int lo = threadIdx.x * per;
  const int hi = min(n, lo + per);
  int s = 0;
  for (int i = lo; i < hi; ++i) s += src[i];
  int total;
  int run = block_exclusive_scan(s, &total);
  for (int i = lo; i < hi; ++i) {
    const int v = src[i];
    dst[i] = run;
    run += v;
  }
  __syncthreads();
  return total;
}

// ------------------------------------------------------------ phases


constexpr int kLdsCols = 4096;  // columns counted in LDS before one global add per block and column

// One LDS pool shared by the binning phases (a phase ends with a block
// barrier before the next one reuses it).
__device__ inline int* lds_pool() {
  __shared__ int pool[2 * kLdsCols];
  return pool;
}

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ void ph_bin(const Dev& d, const double* __restrict__ pos) {
  int* lcnt = lds_pool();
  const bool lds = d.n_cols <= kLdsCols;
  if (lds)
    for (int c = threadIdx.x; c < d.n_cols; c += blockDim.x) lcnt[c] = 0;
  __syncthreads();
  for (int a = gtid(); a < d.n_atoms; a += gthreads()) {
    const GridInfo gi = d.grids[d.atom_grid[a]];
    const ReplicaInfo& rp = d.reps[gi.replica];
    double w[3];
    for (int k = 0; k < 3; ++k) {
      const double x = pos[3 * a + k];
      d.x_build[3 * a + k] = x;
      w[k] = wrap_canon(x, rp.box[k]);
      d.xw[3 * a + k] = w[k];
    }
    int cx = (int)(w[0] / gi.wx), cy = (int)(w[1] / gi.wy);
    cx = cx < 0 ? 0 : (cx >= gi.ncx ? gi.ncx - 1 : cx);
    cy = cy < 0 ? 0 : (cy >= gi.ncy ? gi.ncy - 1 : cy);
    const int col = gi.col_base + cx + gi.ncx * cy;
    d.atom_col[a] = col;
    if (lds) atomicAdd(&lcnt[col], 1);
    else atomicAdd(&d.col_count[col], 1);
  }
  __syncthreads();
  if (lds)
    for (int c = threadIdx.x; c < d.n_cols; c += blockDim.x)
      if (lcnt[c]) atomicAdd(&d.col_count[c], lcnt[c]);
  __syncthreads();
}

// One block: column offsets, SC allocation per column, SC table.
__device__ void ph_scan_cols(const Dev& d) {
  const int C = d.n_cols;
  block_scan_array(d.col_count, d.col_start, C);
  for (int c = threadIdx.x; c < C; c += blockDim.x) d.col_nsc[c] = (d.col_count[c] + kSc - 1) / kSc;
  __syncthreads();
  block_scan_array(d.col_nsc, d.col_fill, C);  // global prefix of SC counts (col_fill as scratch)
  for (int s = threadIdx.x; s < d.sc_cap; s += blockDim.x) d.sc_n[s] = 0;
  __syncthreads();
  for (int c = threadIdx.x; c < C; c += blockDim.x) {
    const GridInfo gi = d.grids[d.col_grid[c]];
    const int within = d.col_fill[c] - d.col_fill[gi.col_base];
    const int nsc = d.col_nsc[c];
    const int s0 = gi.sc_base + within;
    if (within + nsc > gi.sc_cap) {  // excluded by the planner's bound; keep the device safe
      atomicOr(d.flags, 16u);
      d.col_nsc[c] = 0;
      d.col_sc[c] = gi.sc_base;
      continue;
    }
    d.col_sc[c] = s0;
    for (int t = 0; t < nsc; ++t) {
      d.sc_first[s0 + t] = d.col_start[c] + kSc * t;
      d.sc_n[s0 + t] = min(kSc, d.col_count[c] - kSc * t);
      d.sc_col[s0 + t] = c;
    }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < C; c += blockDim.x) d.col_fill[c] = 0;
}

// Atoms into their column's bucket (order inside a bucket is arbitrary; the
// rank sort fixes it).  Each block reserves one range per column.
__device__ void ph_scatter(const Dev& d) {
  int* lcnt = lds_pool();
  int* lbase = lcnt + kLdsCols;
  const bool lds = d.n_cols <= kLdsCols;
  if (!lds) {
    for (int a = gtid(); a < d.n_atoms; a += gthreads()) {
      const int col = d.atom_col[a];
      const int p = d.col_start[col] + atomicAdd(&d.col_fill[col], 1);
      d.bucket[p] = a;
      d.bucket_z[p] = d.xw[3 * a + 2];
    }
    return;
  }
  for (int c = threadIdx.x; c < d.n_cols; c += blockDim.x) lcnt[c] = 0;
  __syncthreads();
  for (int a = gtid(); a < d.n_atoms; a += gthreads()) atomicAdd(&lcnt[d.atom_col[a]], 1);
  __syncthreads();
  for (int c = threadIdx.x; c < d.n_cols; c += blockDim.x) {
    lbase[c] = lcnt[c] ? d.col_start[c] + atomicAdd(&d.col_fill[c], lcnt[c]) : 0;
    lcnt[c] = 0;
  }
  __syncthreads();
  for (int a = gtid(); a < d.n_atoms; a += gthreads()) {
    const int col = d.atom_col[a];
    const int p = lbase[col] + atomicAdd(&lcnt[col], 1);
    d.bucket[p] = a;
    d.bucket_z[p] = d.xw[3 * a + 2];
  }
  __syncthreads();
}

// Rank sort of each column by (wrapped z, atom index).  One wave per 64
// bucket positions of a column (the column's future SCs): each lane counts
// the column's atoms that precede its own, the column streamed through a
// 64-entry LDS window with the next window prefetched into registers.
__device__ void ph_sort_cols(const Dev& d) {
  __shared__ double kz[kBlk];
  __shared__ int ka[kBlk];
  const int lane = threadIdx.x & 63;
  double* wz = kz + (threadIdx.x & ~63);
  int* wa = ka + (threadIdx.x & ~63);
  for (int s = gwave(); s < d.sc_cap; s += gwaves()) {
    const int n_i = d.sc_n[s];
    if (n_i == 0) continue;
    const int c = d.sc_col[s];
    const int base = d.col_start[c], n = d.col_count[c];
    const bool have = lane < n_i;
    const int p = d.sc_first[s] + lane;
    const int ai = have ? d.bucket[p] : 0;
    const double zi = have ? d.bucket_z[p] : 0.0;
    int aj = lane < n ? d.bucket[base + lane] : 0;
    double zj = lane < n ? d.bucket_z[base + lane] : 0.0;
    int rank = 0;
    for (int jb = 0; jb < n; jb += 64) {
      wave_sync();
      wz[lane] = zj;
      wa[lane] = aj;
      wave_sync();
      const int jn = jb + 64 + lane;
      aj = jn < n ? d.bucket[base + jn] : 0;
      zj = jn < n ? d.bucket_z[base + jn] : 0.0;
      const int m = min(64, n - jb);
      int j = 0;
      for (; j + 8 <= m; j += 8) {
        double zz[8];
        int aa[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          zz[u] = wz[j + u];
          aa[u] = wa[j + u];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) rank += (zz[u] < zi || (zz[u] == zi && aa[u] < ai)) ? 1 : 0;
      }
      for (; j < m; ++j) rank += (wz[j] < zi || (wz[j] == zi && wa[j] < ai)) ? 1 : 0;
    }
    if (have) d.sorted[base + rank] = ai;
  }
}

// rank of this lane's key among the lanes of its group (ties by atom index)
__device__ inline int group_rank(double key, int atom, int grp) {
  int r = 0;
  for (int j = 0; j < 64; ++j) {
    const double kj = __shfl(key, j);
    const int aj = __shfl(atom, j);
    const int gj = __shfl(grp, j);
    r += (gj == grp && (kj < key || (kj == key && aj < atom))) ? 1 : 0;
  }
  return r;
}

__device__ inline double wave_min8(double v) {
  v = fmin(v, __shfl_xor(v, 1));
  v = fmin(v, __shfl_xor(v, 2));
  return fmin(v, __shfl_xor(v, 4));
}
__device__ inline double wave_max8(double v) {
  v = fmax(v, __shfl_xor(v, 1));
  v = fmax(v, __shfl_xor(v, 2));
  return fmax(v, __shfl_xor(v, 4));
}
__device__ inline double wave_minall(double v) {
  for (int o = 8; o < 64; o <<= 1) v = fmin(v, __shfl_xor(v, o));
  return v;
}
__device__ inline double wave_maxall(double v) {
  for (int o = 8; o < 64; o <<= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

// One wave per super-cluster: 2x2x2 split of a full SC (x halves, then y
// halves, then z clusters of 8), slot tables, per-slot parameters, boxes.
__device__ void ph_build_sc(const Dev& d) {
  const int l = threadIdx.x & 63;
  for (int s = gwave(); s < d.sc_cap; s += gwaves()) {
    const int n = d.sc_n[s];
    const bool have = l < n;
    int a = have ? d.sorted[d.sc_first[s] + l] : -1;
    double w[3] = {0, 0, 0};
    if (have)
      for (int k = 0; k < 3; ++k) w[k] = d.xw[3 * a + k];
    int target = l;  // slot of this lane's atom
    if (n == kSc) {
      const int rx = group_rank(w[0], a, 0);
      const int hx = rx >> 5;
      const int ry = group_rank(w[1], a, hx);
      const int q = hx * 2 + (ry >> 4);
      const int rz = group_rank(w[2], a, q);
      target = (q * 2 + (rz >> 3)) * kCl + (rz & 7);
    }
    // forward permutation inside the wave (a bijection of the 64 lanes)
    const int addr = target * 4;
    a = __builtin_amdgcn_ds_permute(addr, a);
    for (int k = 0; k < 3; ++k) {
      const long long bits = __double_as_longlong(w[k]);
      const int lo = __builtin_amdgcn_ds_permute(addr, (int)(bits & 0xffffffffll));
      const int hi = __builtin_amdgcn_ds_permute(addr, (int)(bits >> 32));
      w[k] = __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
    }
    const int sl = s * kSc + l;
    d.slot_atom[sl] = a;
    d.slot_xw[sl] = make_double4(w[0], w[1], w[2], 0.0);
    d.slot_comp[sl] = a >= 0 ? d.atom_comp[a] : -1;
    d.slot_type[sl] = a >= 0 ? d.atom_type[a] : 0;
    if (a >= 0) {
      d.atom_slot[a] = sl;
      const int t = d.atom_type[a];
      const double sg = d.type_sigma[t], ep = d.type_eps[t], qq = d.type_q[t];
      const double sh = 0.5 * sg, e2 = 2.0 * sqrt(ep), qs = qq * sqrt(kKe);
      d.se32[sl] = make_float2((float)sh, (float)e2);
      d.se64[sl] = make_double2(sh, e2);
      d.q32[sl] = (float)qs;
      d.q64[sl] = qs;
    } else {
      d.se32[sl] = make_float2(0.f, 0.f);
      d.se64[sl] = make_double2(0.0, 0.0);
      d.q32[sl] = 0.f;
      d.q64[sl] = 0.0;
    }
    // boxes over valid slots
    const bool v = a >= 0;
    double lo[3], hi[3];
    for (int k = 0; k < 3; ++k) {
      lo[k] = v ? w[k] : 1e300;
      hi[k] = v ? w[k] : -1e300;
    }
    double clo[3], chi[3], slo[3], shi[3];
    for (int k = 0; k < 3; ++k) {
      clo[k] = wave_min8(lo[k]);
      chi[k] = wave_max8(hi[k]);
      slo[k] = wave_minall(clo[k]);
      shi[k] = wave_maxall(chi[k]);
    }
    int cnt = v ? 1 : 0;
    cnt += __shfl_xor(cnt, 1);
    cnt += __shfl_xor(cnt, 2);
    cnt += __shfl_xor(cnt, 4);
    if ((l & 7) == 0) {
      const int c = s * kScCl + (l >> 3);
      d.cl_n[c] = cnt;
      for (int k = 0; k < 3; ++k) {
        d.cl_bbox[c * 6 + k] = cnt ? clo[k] : 0.0;
        d.cl_bbox[c * 6 + 3 + k] = cnt ? chi[k] : 0.0;
      }
    }
    double org[3];
    for (int k = 0; k < 3; ++k) {
      const double a0 = n ? slo[k] : 0.0, a1 = n ? shi[k] : 0.0;
      org[k] = 0.5 * (a0 + a1);
      if (l == 0) {
        d.sc_bbox[s * 6 + k] = a0;
        d.sc_bbox[s * 6 + 3 + k] = a1;
        d.sc_origin[s * 3 + k] = org[k];
      }
    }
    // coordinates relative to the SC origin for the first evaluation on
    // this list (the positions are those of the build), and cleared force
    // accumulators; later calls refresh them in the prepare pass
    double q[3] = {0.0, 0.0, 0.0};
    if (v) {
      for (int k = 0; k < 3; ++k) q[k] = w[k] - org[k];
      // what the per-call pass adds to the displacement since the build,
      // and the slot + 1 (0 = never placed)
      d.atom_off[a] = make_double4(q[0], q[1], q[2], (double)(sl + 1));
      d.atom_box[a] = d.sc_box[s];
    }
    d.pos32[sl] = make_float4((float)q[0], (float)q[1], (float)q[2], d.q32[sl]);
    d.pos64[sl] = make_double4(q[0], q[1], q[2], d.q64[sl]);
    const int slots = d.sc_cap * kSc;
    d.ffix[sl] = 0ull;
    d.ffix[slots + sl] = 0ull;
    d.ffix[2 * slots + sl] = 0ull;
  }
}

__device__ inline double gap1(double ilo, double ihi, double jlo, double jhi) {
  return fmax(0.0, fmax(jlo - ihi, ilo - jhi));
}

// Cluster-pair search, kStrips waves per i-SC: the neighbour columns that
// pass the x-y test are dealt round-robin to the waves of the SC.  Each wave
// walks its candidates in a fixed order: j-grid, x shift and column, y shift
// and column, j-SC in z order, z shift, then j-cluster; its entries follow
// those of the SC's lower strips.  WRITE = false counts, true writes.
template <bool WRITE>
__device__ void ph_search(const Dev& d, double rlm) {
  const double rl2 = rlm * rlm;
  const int lane = threadIdx.x & 63;
  const int ic = lane >> 3, jcq = lane & 7;  // search layout: (i-cluster, j-cluster)
  for (int sw = gwave(); sw < d.sc_cap * kStrips; sw += gwaves()) {
    const int s = sw / kStrips, strip = sw % kStrips;
    if (d.sc_n[s] == 0) {
      if (!WRITE && lane == 0) d.strip_count[sw] = 0;
      continue;
    }
    const GridInfo gi = d.grids[d.col_grid[d.sc_col[s]]];
    const ReplicaInfo rp = d.reps[gi.replica];
    const double L[3] = {rp.box[0], rp.box[1], rp.box[2]};
    double ilo[3], ihi[3], cilo[3], cihi[3];
    const int icl = s * kScCl + ic;
    const bool i_ok = d.cl_n[icl] > 0;
    for (int k = 0; k < 3; ++k) {
      ilo[k] = d.sc_bbox[s * 6 + k];
      ihi[k] = d.sc_bbox[s * 6 + 3 + k];
      cilo[k] = d.cl_bbox[icl * 6 + k];
      cihi[k] = d.cl_bbox[icl * 6 + 3 + k];
    }
    int count = 0, n_col = 0;
    const int wbase = WRITE ? d.strip_start[sw] : 0;
    for (int gj_idx = rp.grid0; gj_idx < rp.grid0 + rp.n_grids; ++gj_idx) {
      const GridInfo gj = d.grids[gj_idx];
      if (gj.n_atoms == 0 || gj.sc_base + gj.sc_cap <= s) continue;
      const int kind = (gi.is_solute && gj.is_solute) ? KIND_SOLU
                       : ((!gi.is_solute && !gj.is_solute) ? KIND_SOLV : KIND_ALCH);
      for (int sxi = -1; sxi <= 1; ++sxi)
        for (int cx = 0; cx < gj.ncx; ++cx) {
          const double xlo = cx * gj.wx + sxi * L[0], xhi = xlo + gj.wx;
          const double gx = gap1(ilo[0], ihi[0], xlo, xhi);
          if (gx >= rlm) continue;
          for (int syi = -1; syi <= 1; ++syi)
            for (int cy = 0; cy < gj.ncy; ++cy) {
              const double ylo = cy * gj.wy + syi * L[1], yhi = ylo + gj.wy;
              const double gy = gap1(ilo[1], ihi[1], ylo, yhi);
              if (gx * gx + gy * gy >= rl2) continue;
              if (n_col++ % kStrips != strip) continue;
              const int col = gj.col_base + cx + gj.ncx * cy;
              const int jsb = max(d.col_sc[col], s), jse = d.col_sc[col] + d.col_nsc[col];
              const int m = (jse - jsb) * 3;  // candidates (j-SC, z shift), j-SC major
              for (int k0 = 0; k0 < m; k0 += 64) {
                // lane-parallel super-cluster box test
                const int k = k0 + lane;
                bool pass = false;
                if (k < m) {
                  const int js = jsb + k / 3, szi = k % 3 - 1;
                  const double sh[3] = {sxi * L[0], syi * L[1], szi * L[2]};
                  double g2 = 0;
                  for (int q = 0; q < 3; ++q) {
                    const double g = gap1(ilo[q], ihi[q], d.sc_bbox[js * 6 + q] + sh[q], d.sc_bbox[js * 6 + 3 + q] + sh[q]);
                    g2 += g * g;
                  }
                  pass = g2 < rl2;
                }
                unsigned long long P = __ballot(pass);
                while (P) {
                  const int b = __ffsll((long long)P) - 1;
                  P &= P - 1;
                  const int js = jsb + (k0 + b) / 3, szi = (k0 + b) % 3 - 1;
                  const double sh[3] = {sxi * L[0], syi * L[1], szi * L[2]};
                  // cluster level: lane (ic, jcq)
                  const int jcl = js * kScCl + jcq;
                  bool ok = i_ok && d.cl_n[jcl] > 0 && jcl >= icl;
                  if (ok) {
                    double c2 = 0;
                    for (int q = 0; q < 3; ++q) {
                      const double g = gap1(cilo[q], cihi[q], d.cl_bbox[jcl * 6 + q] + sh[q],
                                            d.cl_bbox[jcl * 6 + 3 + q] + sh[q]);
                      c2 += g * g;
                    }
                    ok = c2 < rl2;
                  }
                  const unsigned long long M = __ballot(ok);
                  if (M == 0) continue;
                  // lane j (0..7) gathers the i-cluster mask of j-cluster j
                  uint32_t imask = 0;
                  for (int bb = 0; bb < kScCl; ++bb) imask |= (uint32_t)((M >> (bb * 8 + (lane & 7))) & 1ull) << bb;
                  const bool emit = lane < 8 && imask != 0;
                  const unsigned long long E = __ballot(emit);
                  if (WRITE && emit) {
                    const int pre = __popcll(E & ((1ull << lane) - 1ull));
                    const int e = wbase + count + pre;
                    if (e < d.ent_cap) {
                      d.ent_jc[e] = js * kScCl + lane;
                      d.ent_info[e] = ent_pack(imask, (uint32_t)kind,
                                               (uint32_t)((sxi + 1) + 3 * (syi + 1) + 9 * (szi + 1)));
                      d.ent_isc[e] = s;
                    }
                  }
                  count += __popcll(E);
                }
              }
            }
        }
    }
    if (!WRITE && lane == 0) d.strip_count[sw] = count;
  }
}

// One block: entry offsets per search strip and per SC, capacity check.
__device__ void ph_scan_entries(const Dev& d) {
  const int total = block_scan_array(d.strip_count, d.strip_start, d.sc_cap * kStrips);
  for (int s = threadIdx.x; s < d.sc_cap; s += blockDim.x) {
    int c = 0;
    for (int p = 0; p < kStrips; ++p) c += d.strip_count[s * kStrips + p];
    d.sc_ecount[s] = c;
    d.sc_estart[s] = d.strip_start[s * kStrips];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    d.ctr[CTR_TILES] = 0;  // summed by the mask phase
    d.ctr[CTR_ENT_NEED] = total;
    if (total > d.ent_cap) atomicOr(d.flags, 16u);
    d.ctr[CTR_NENT] = total > d.ent_cap ? 0 : total;
  }
  __syncthreads();
}

// Work units, after the mask pass, in three passes.  A unit is a run of
// one SC's entries, cut greedily where it would exceed epu entries or, past
// its first entry, tcap tiles (the pruned masks' counts; a solute-solvent
// tile, fed from FP64 data and the type-pair table, counts kAlchTileCost).

__device__ inline bool entry_is_alch(uint32_t info) { return ((info >> 8) & 3u) == KIND_ALCH; }
__device__ inline int entry_cost_tiles(uint32_t info) {
  const int t = __popc(info & 0xffu);
  return entry_is_alch(info) ? kAlchTileCost * t : t;
}

// Pass A, one wave per SC: the greedy cuts (scalar, over each 64-entry
// chunk), marked with kUnitStart in ent_info; unit count per SC.
__device__ void ph_units_count(const Dev& d, int epu, int tcap) {
  const int lane = threadIdx.x & 63;
  const bool ok_all = d.ctr[CTR_NENT] == d.ctr[CTR_ENT_NEED];
  for (int s = gwave(); s < d.sc_cap; s += gwaves()) {
    const int cnt = ok_all ? d.sc_ecount[s] : 0;
    const int e0 = d.sc_estart[s];
    int nu = 0, ne = 0, nt = 0;
    for (int base = 0; base < cnt; base += 64) {
      const int e = e0 + base + lane;
      const bool valid = base + lane < cnt;
      const uint32_t info = valid ? d.ent_info[e] : 0u;
      const int t = entry_cost_tiles(info);
      const int m = min(64, cnt - base);
      unsigned long long start = 0;
      for (int l = 0; l < m; ++l) {
        const int tl = __builtin_amdgcn_readlane(t, l);
        if (ne == 0 || ne == epu || nt + tl > tcap) {
          start |= 1ull << l;
          ++nu;
          ne = 0;
          nt = 0;
        }
        ++ne;
        nt += tl;
      }
      if (valid) d.ent_info[e] = (info & ~kUnitStart) | (((start >> lane) & 1ull) ? kUnitStart : 0u);
    }
    if (lane == 0) d.sc_ustart[s] = nu;
  }
}

// Pass B, one block: offsets of each SC's units, counters, replica ranges.
__device__ void ph_units_scan(const Dev& d) {
  const int n = d.sc_cap;
  const int total = block_scan_array(d.sc_ustart, d.sc_ustart, n);
  const bool fits = total <= d.unit_cap;
  if (threadIdx.x == 0) {
    d.ctr[CTR_UNIT_NEED] = total;
    d.ctr[CTR_NUNIT] = fits ? total : 0;
    if (!fits) atomicOr(d.flags, 16u);
  }
  for (int k = threadIdx.x; k <= d.n_reps; k += blockDim.x) {
    int v;
    if (!fits) v = 0;
    else if (k == d.n_reps) v = total;
    else v = d.reps[k].sc_begin < n ? d.sc_ustart[d.reps[k].sc_begin] : total;
    d.rep_ustart[k] = v;
  }
  __syncthreads();
}

// Pass C, one wave per SC: the unit table (a unit ends where the next one
// starts, the last at the SC's end).
__device__ void ph_units_fill(const Dev& d) {
  const int lane = threadIdx.x & 63;
  if (d.ctr[CTR_UNIT_NEED] > d.unit_cap) return;
  const bool ok_all = d.ctr[CTR_NENT] == d.ctr[CTR_ENT_NEED];
  int* ucol = reinterpret_cast<int*>(d.units);
  for (int s = gwave(); s < d.sc_cap; s += gwaves()) {
    const int cnt = ok_all ? d.sc_ecount[s] : 0;
    if (cnt == 0) continue;
    const int e0 = d.sc_estart[s], u0 = d.sc_ustart[s];
    const GridInfo g = d.grids[d.col_grid[d.sc_col[s]]];
    const int rep = g.replica | (g.is_solute ? kUnitSolute : 0);
    int u = u0;
    const unsigned long long below = (1ull << lane) - 1ull;
    for (int base = 0; base < cnt; base += 64) {
      const int e = e0 + base + lane;
      const bool valid = base + lane < cnt;
      const uint32_t info = valid ? d.ent_info[e] : 0u;
      const bool st = valid && (info & kUnitStart);
      const unsigned long long S = __ballot(st);
      if (st) {
        const int idx = u + __popcll(S & below);
        ucol[4 * idx + 0] = s;
        ucol[4 * idx + 1] = e;
        ucol[4 * idx + 3] = rep;
        if (idx > u0) ucol[4 * (idx - 1) + 2] = e;  // the previous unit ends here
      }
      u += __popcll(S);
    }
    if (lane == 0) ucol[4 * (u - 1) + 2] = e0 + cnt;
  }
}

// Start records of the tile launch's nw waves (equal runs of units): the
// run, whether it holds solute units, and the first unit's header and
// entry data, so that a wave's first loads need neither the unit count nor
// the unit table.  One wave per record.
__device__ void ph_wave_records(const Dev& d, int nw) {
  const int lane = threadIdx.x & 63;
  const int n = d.ctr[CTR_NUNIT];
  for (int w = gwave(); w < nw; w += gwaves()) {
    const int ub = (int)((long long)n * w / nw);
    const int nr = (int)((long long)n * (w + 1) / nw) - ub;
    bool sol = false;
    for (int r = lane; r < nr; r += 64) sol = sol || (d.units[ub + r].w & kUnitSolute) != 0;
    const bool any_sol = __ballot(sol) != 0ull;
    const int4 U0 = nr > 0 ? d.units[ub] : make_int4(0, 0, 0, 0);
    if (lane == 0) {
      d.wrec[w] = make_int4(ub, nr, any_sol ? 1 : 0, 0);
      d.wrec_u0[w] = U0;
    }
    if (lane < kMaxEpu) {
      const int e = U0.y + lane;
      int jc = 0;
      uint32_t inf = 0u;
      double4 off = make_double4(0.0, 0.0, 0.0, 0.0);
      if (nr > 0 && e < U0.z) {
        jc = d.ent_jc[e];
        inf = d.ent_info[e];
        off = d.ent_off[e];
      }
      d.wrec_jc[w * kMaxEpu + lane] = jc;
      d.wrec_info[w * kMaxEpu + lane] = inf;
      d.wrec_off[w * kMaxEpu + lane] = off;
    }
  }
  if (gtid() == 0) d.ctr[CTR_WAVES] = nw;
}

__device__ inline bool is_excluded(const Dev& d, int a, int b) {
  const int lo = a < b ? a : b, hi = a < b ? b : a;
  int l = d.excl_start[lo], r = d.excl_start[lo + 1];
  while (l < r) {
    const int m = (l + r) >> 1;
    const int v = d.excl_j[m];
    if (v == hi) return true;
    if (v < hi) l = m + 1;
    else r = m;
  }
  return false;
}

// Atom-pair masks of each entry; lane = jl * 8 + il (the tile kernel's
// layout).  A bit is set for a valid, non-excluded pair (i<j inside one
// cluster) whose build-time distance in this entry's image is below the list
// radius; i-clusters left without any pair are dropped from the entry.
__device__ void ph_masks(const Dev& d, double rl2) {
  const int lane = threadIdx.x & 63;
  const int il = lane & 7, jl = lane >> 3;
  const int n_ent = d.ctr[CTR_NENT];
  int tiles = 0;  // 64-lane pair tiles of this wave's entries
  for (int e = gwave(); e < n_ent; e += gwaves()) {
    const int s = d.ent_isc[e];
    const int jc = d.ent_jc[e];
    const uint32_t info = d.ent_info[e];
    const uint32_t imask = info & 0xffu;
    const int code = (int)((info >> 16) & 31u);
    const int jsl = jc * kCl + jl;
    const int cj = d.slot_comp[jsl];
    const double4 wj = d.slot_xw[jsl];
    const double4 L = d.sc_box[s];
    const double shx = (code % 3 - 1) * L.x, shy = ((code / 3) % 3 - 1) * L.y, shz = (code / 9 - 1) * L.z;
    const double xj = wj.x + shx, yj = wj.y + shy, zj = wj.z + shz;
    bool ok[kScCl];
    // independent loads for all i-clusters first, exclusion searches only
    // for pairs inside one exclusion component
#pragma unroll
    for (int c = 0; c < kScCl; ++c) {
      const int isl = (s * kScCl + c) * kCl + il;
      const int ci = d.slot_comp[isl];
      const double4 wi = d.slot_xw[isl];
      const double vx = xj - wi.x, vy = yj - wi.y, vz = zj - wi.z;
      const double r2 = vx * vx + vy * vy + vz * vz;
      ok[c] = (imask & (1u << c)) && ci >= 0 && cj >= 0 && (s * kScCl + c != jc || il < jl) && r2 < rl2;
      if (ok[c] && ci == cj) ok[c] = !is_excluded(d, d.slot_atom[isl], d.slot_atom[jsl]);
    }
    uint32_t keep = 0;
    unsigned long long mine = 0;
#pragma unroll
    for (int c = 0; c < kScCl; ++c) {
      const unsigned long long M = __ballot(ok[c]);
      if (M) keep |= 1u << c;
      if (lane == c) mine = M;
    }
    if (lane < kScCl) d.ent_mask[(size_t)e * kScCl + lane] = mine;
    if (lane == 0) {
      // the tile kernel adds this to the j-cluster's local coordinates
      const int sj = jc >> 3;
      d.ent_off[e] = make_double4(d.sc_origin[3 * sj] + shx - d.sc_origin[3 * s],
                                  d.sc_origin[3 * sj + 1] + shy - d.sc_origin[3 * s + 1],
                                  d.sc_origin[3 * sj + 2] + shz - d.sc_origin[3 * s + 2], 0.0);
    }
    if (lane == 0 && keep != imask) d.ent_info[e] = (info & ~0xffu) | keep;
    tiles += __popc(keep);
  }
  // one counter update per wave: a single contended address would
  // serialise tens of thousands of atomics
  if (lane == 0 && tiles) atomicAdd(&d.ctr[CTR_TILES], tiles);
}

// Column counters start at zero for the next build (the workspace is
// cleared when it is bound, so the first build finds them zero too).
__device__ void ph_end(const Dev& d) {
  for (int c = gtid(); c < d.n_cols; c += gthreads()) d.col_count[c] = 0;
  if (gtid() == 0) {
    d.ctr[CTR_NBUILD] += 1;
    __atomic_store_n(d.rebuild, 0, __ATOMIC_RELAXED);
  }
}

// ------------------------------------------------------------ kernels

#define GATED if (!rebuild_on(d)) return
__global__ void __launch_bounds__(kBlk) k_bin(Dev d, const double* pos) { GATED; ph_bin(d, pos); }
__global__ void __launch_bounds__(kBlk) k_scan_cols(Dev d) { GATED; ph_scan_cols(d); }
__global__ void __launch_bounds__(kBlk) k_scatter(Dev d) { GATED; ph_scatter(d); }
__global__ void __launch_bounds__(kBlk) k_sort_cols(Dev d) { GATED; ph_sort_cols(d); }
__global__ void __launch_bounds__(kBlk) k_build_sc(Dev d) { GATED; ph_build_sc(d); }
__global__ void __launch_bounds__(kBlk) k_search_count(Dev d, double rlm) { GATED; ph_search<false>(d, rlm); }
__global__ void __launch_bounds__(kBlk) k_scan_entries(Dev d) { GATED; ph_scan_entries(d); }
__global__ void __launch_bounds__(kBlk) k_search_write(Dev d, double rlm) { GATED; ph_search<true>(d, rlm); }
__global__ void __launch_bounds__(kBlk) k_units_count(Dev d, int epu, int tcap, int force) {
  if (!force) { GATED; }
  ph_units_count(d, epu, tcap);
}
__global__ void __launch_bounds__(kBlk) k_units_scan(Dev d, int force) {
  if (!force) { GATED; }
  ph_units_scan(d);
}
__global__ void __launch_bounds__(kBlk) k_units_fill(Dev d, int force) {
  if (!force) { GATED; }
  ph_units_fill(d);
}
__global__ void __launch_bounds__(kBlk) k_wave_records(Dev d, int nw, int force) {
  if (!force && !rebuild_on(d)) return;
  ph_wave_records(d, nw);
}
__global__ void __launch_bounds__(kBlk) k_masks(Dev d, double rl2) { GATED; ph_masks(d, rl2); }
__global__ void __launch_bounds__(kBlk) k_end(Dev d) { GATED; ph_end(d); }
#undef GATED

static inline int clampi(long long v, int lo, int hi) { return (int)(v < lo ? lo : (v > hi ? hi : v)); }

// Grid barrier for the fused list build.  Every wave waits for its own
// stores, then one thread per block writes back its XCD's L2 and arrives on
// one of eight group counters (blocks b = g mod 8); the last block of a
// group arrives on the top counter, and the last group's block runs the
// optional one-block section SERIAL (a scan) before it opens the next
// generation.  Waiters poll the generation with relaxed loads and acquire
// once.  The wait is bounded: a block that gives up raises
// ALCH_NB_FLAG_BARRIER_TIMEOUT and proceeds, so every wave finishes.  The
// grid is sized on the host to fit the device at once.
template <class Serial>
__device__ inline void grid_barrier(const Dev& d, unsigned int& gen, Serial serial) {
  __shared__ int is_last;
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  unsigned int* bar = d.barrier;
  if (threadIdx.x == 0) {
    const unsigned int grp = blockIdx.x % kBarGroups;
    const unsigned int n_grp = (gridDim.x - grp + kBarGroups - 1) / kBarGroups;
    const unsigned int n_top = min(gridDim.x, (unsigned int)kBarGroups);
    int last = 0;
    unsigned int* gc = bar + kBarStride * (grp + 1);
    // the arrival publishes the block's writes (release: one L2 write-back);
    // what the block reads next is acquired by the top-level arrival (the
    // last block) or by the acquire after the wait (all others)
    if (__hip_atomic_fetch_add(gc, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT) == n_grp - 1) {
      __hip_atomic_store(gc, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      last = __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == n_top - 1;
    }
    is_last = last;
  }
  __syncthreads();
  if (is_last) {
    serial();
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
      __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&bar[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
  } else if (threadIdx.x == 0) {
    unsigned int spins = 0;
    while (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
      __builtin_amdgcn_s_sleep(2);
      if (++spins > (1u << 24)) {
        atomicOr(d.flags, 32u);
        break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  gen += 1;
  __syncthreads();
}

// The whole list build in one launch (phases separated by grid barriers;
// the one-block scans run inside the barriers).
__global__ void __launch_bounds__(kBlk) k_list_fused(Dev d, const double* __restrict__ pos, double rlm, double rl2,
                                                     int epu, int tcap, int nw) {
  if (!rebuild_on(d)) return;
  __shared__ unsigned int gen_s;
  if (threadIdx.x == 0) gen_s = __hip_atomic_load(&d.barrier[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  unsigned int gen = gen_s;
  auto none = [] {};
  ph_bin(d, pos);
  grid_barrier(d, gen, [&] { ph_scan_cols(d); });
  ph_scatter(d);
  grid_barrier(d, gen, none);
  ph_sort_cols(d);
  grid_barrier(d, gen, none);
  ph_build_sc(d);
  grid_barrier(d, gen, none);
  ph_search<false>(d, rlm);
  grid_barrier(d, gen, [&] { ph_scan_entries(d); });
  ph_search<true>(d, rlm);
  grid_barrier(d, gen, none);
  ph_masks(d, rl2);
  grid_barrier(d, gen, none);
  ph_units_count(d, epu, tcap);
  grid_barrier(d, gen, [&] { ph_units_scan(d); });
  ph_units_fill(d);
  grid_barrier(d, gen, none);
  ph_wave_records(d, nw);
  grid_barrier(d, gen, none);
  ph_end(d);
}

hipError_t launch_list_build(const Dev& d, hipStream_t st, const double* pos, double r_list, const TileShape& sh,
                             int fused_blocks) {
  const int epu = sh.epu, tcap = sh.tiles;
  const double rlm = r_list * (1.0 + 1e-12) + 1e-9;  // conservative box test
  const double rl2 = rlm * rlm;  // masks keep the same margin; the export test is exact
  const dim3 B(kBlk);
  if (fused_blocks > 0) {
    hipLaunchKernelGGL(k_list_fused, dim3(fused_blocks), B, 0, st, d, pos, rlm, rl2, epu, tcap, 4 * sh.blocks);
    return hipGetLastError();
  }
  const int g_atoms = clampi((d.n_atoms + kBlk - 1) / kBlk, 1, 256);
  const int g_sc = clampi((d.sc_cap + kWpb - 1) / kWpb, 1, 256);
  const int g_srch = clampi((d.sc_cap * kStrips + kWpb - 1) / kWpb, 1, 512);
  const int g_ent = clampi(((long long)d.ent_cap + kWpb - 1) / kWpb, 1, 256);
  hipLaunchKernelGGL(k_bin, dim3(g_atoms), B, 0, st, d, pos);
  hipLaunchKernelGGL(k_scan_cols, dim3(1), B, 0, st, d);
  hipLaunchKernelGGL(k_scatter, dim3(g_atoms), B, 0, st, d);
  hipLaunchKernelGGL(k_sort_cols, dim3(g_sc), B, 0, st, d);
  hipLaunchKernelGGL(k_build_sc, dim3(g_sc), B, 0, st, d);
  hipLaunchKernelGGL(k_search_count, dim3(g_srch), B, 0, st, d, rlm);
  hipLaunchKernelGGL(k_scan_entries, dim3(1), B, 0, st, d);
  hipLaunchKernelGGL(k_search_write, dim3(g_srch), B, 0, st, d, rlm);
  hipLaunchKernelGGL(k_masks, dim3(g_ent), B, 0, st, d, rl2);
  hipLaunchKernelGGL(k_units_count, dim3(g_sc), B, 0, st, d, epu, tcap, 0);
  hipLaunchKernelGGL(k_units_scan, dim3(1), B, 0, st, d, 0);
  hipLaunchKernelGGL(k_units_fill, dim3(g_sc), B, 0, st, d, 0);
  hipLaunchKernelGGL(k_wave_records, dim3(clampi((4 * sh.blocks + kWpb - 1) / kWpb, 1, 256)), B, 0, st, d,
                     4 * sh.blocks, 0);
  hipLaunchKernelGGL(k_end, dim3(1), dim3(64), 0, st, d);
  return hipGetLastError();
}

int list_fused_max_blocks() {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k_list_fused), kBlk, 0) !=
      hipSuccess)
    return 0;
  return per_cu;
}

hipError_t launch_units(const Dev& d, hipStream_t st, const TileShape& sh) {
  const int g_sc = clampi((d.sc_cap + kWpb - 1) / kWpb, 1, 256);
  hipLaunchKernelGGL(k_units_count, dim3(g_sc), dim3(kBlk), 0, st, d, sh.epu, sh.tiles, 1);
  hipLaunchKernelGGL(k_units_scan, dim3(1), dim3(kBlk), 0, st, d, 1);
  hipLaunchKernelGGL(k_units_fill, dim3(g_sc), dim3(kBlk), 0, st, d, 1);
  hipLaunchKernelGGL(k_wave_records, dim3(clampi((4 * sh.blocks + kWpb - 1) / kWpb, 1, 256)), dim3(kBlk), 0, st, d,
                     4 * sh.blocks, 1);
  return hipGetLastError();
}

// ------------------------------------------------------------ pair export

// Canonical FP64 test of every masked pair of the list at build-time
// positions; a pair is reported from the entry whose image shift equals its
// minimum image, so each pair appears once.
__global__ void __launch_bounds__(kBlk) k_export(Dev d, double rl2, int* __restrict__ out, long long cap,
                                                 unsigned long long* __restrict__ counter) {
#pragma clang fp contract(off)
  const int lane = threadIdx.x & 63;
  const int il = lane & 7, jl = lane >> 3;
  const int n_ent = d.ctr[CTR_NENT];
  int tiles = 0;  // 64-lane pair tiles of this wave's entries
  for (int e = gwave(); e < n_ent; e += gwaves()) {
    const int s = d.ent_isc[e];
    const int jc = d.ent_jc[e];
    const uint32_t info = d.ent_info[e];
    const int code = (int)((info >> 16) & 31u);
    const int shift[3] = {code % 3 - 1, (code / 3) % 3 - 1, code / 9 - 1};
    const int aj = d.slot_atom[jc * kCl + jl];
    for (int c = 0; c < kScCl; ++c) {
      const unsigned long long M = d.ent_mask[(size_t)e * kScCl + c];
      if (!((M >> lane) & 1ull)) continue;
      const int ai = d.slot_atom[(s * kScCl + c) * kCl + il];
      const ReplicaInfo& rp = d.reps[d.grids[d.atom_grid[ai]].replica];
      double dd[3];
      bool img_ok = true;
      for (int k = 0; k < 3; ++k) {
        const double L = rp.box[k];
        const double wi = wrap_canon(d.x_build[3 * ai + k], L);
        const double wj = wrap_canon(d.x_build[3 * aj + k], L);
        const double raw = wj - wi;
        const int m = raw > 0.5 * L ? -1 : (raw < -0.5 * L ? 1 : 0);
        img_ok = img_ok && (m == shift[k]);
        // canonical order: displacement of the higher index from the lower
        const double v = ai < aj ? raw : -raw;
        dd[k] = v > 0.5 * L ? v - L : (v < -0.5 * L ? v + L : v);
      }
      const double r2 = (dd[0] * dd[0] + dd[1] * dd[1]) + dd[2] * dd[2];
      if (img_ok && r2 < rl2) {
        const unsigned long long idx = atomicAdd(counter, 1ull);
        if ((long long)idx < cap) {
          out[2 * idx] = min(ai, aj);
          out[2 * idx + 1] = max(ai, aj);
        }
      }
    }
  }
}

hipError_t launch_export(const Dev& d, hipStream_t st, double r_list, int* out, long long cap,
                         unsigned long long* counter) {
  const int g_ent = clampi(((long long)d.ent_cap + 3) / 4, 1, 4096);
  hipLaunchKernelGGL(k_export, dim3(g_ent), dim3(kBlk), 0, st, d, r_list * r_list, out, cap, counter);
  return hipGetLastError();
}

}  // namespace anb
