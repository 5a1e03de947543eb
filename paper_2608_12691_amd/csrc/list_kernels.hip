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

constexpr int kBlk = 256;

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
  const int t = threadIdx.x;
  buf[t] = v;
  __syncthreads();
  for (int off = 1; off < kBlk; off <<= 1) {
    const int add = t >= off ? buf[t - off] : 0;
    __syncthreads();
    buf[t] += add;
    __syncthreads();
  }
  const int incl = buf[t];
  *total = buf[kBlk - 1];
  __syncthreads();
  return incl - v;
}

// Exclusive scan of src[0..n) into dst by one block; returns the total.
// src and dst may alias (values are read before they are overwritten).
__device__ int block_scan_array(const int* src, int* dst, int n) {
  const int per = (n + kBlk - 1) / kBlk;
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

__device__ void ph_begin(const Dev& d) {
  if (gtid() == 0) d.ctr[CTR_TILES] = 0;
  for (int c = gtid(); c < d.n_cols; c += gthreads()) {
    d.col_count[c] = 0;
    d.col_fill[c] = 0;
  }
}

__device__ void ph_bin(const Dev& d, const double* __restrict__ pos) {
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
    atomicAdd(&d.col_count[col], 1);
  }
}

// Block 0 only: column offsets, SC allocation per column, SC table.
__device__ void ph_scan_cols(const Dev& d) {
  if (blockIdx.x != 0) return;
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

__device__ void ph_scatter(const Dev& d) {
  for (int a = gtid(); a < d.n_atoms; a += gthreads()) {
    const int col = d.atom_col[a];
    const int p = d.col_start[col] + atomicAdd(&d.col_fill[col], 1);
    d.bucket[p] = a;
  }
}

// Rank sort of each column by (wrapped z, atom index); one block per column.
__device__ void ph_sort_cols(const Dev& d) {
  constexpr int CH = 1024;
  __shared__ double kz[CH];
  __shared__ int ka[CH];
  for (int c = blockIdx.x; c < d.n_cols; c += gridDim.x) {
    const int n = d.col_count[c];
    const int base = d.col_start[c];
    for (int ib = 0; ib < n; ib += blockDim.x) {
      const int i = ib + threadIdx.x;
      const bool have = i < n;
      int ai = 0;
      double zi = 0;
      if (have) {
        ai = d.bucket[base + i];
        zi = d.xw[3 * ai + 2];
      }
      int rank = 0;
      for (int jb = 0; jb < n; jb += CH) {
        __syncthreads();
        for (int j = threadIdx.x; j < CH && jb + j < n; j += blockDim.x) {
          const int aj = d.bucket[base + jb + j];
          ka[j] = aj;
          kz[j] = d.xw[3 * aj + 2];
        }
        __syncthreads();
        if (have) {
          const int m = min(CH, n - jb);
          for (int j = 0; j < m; ++j) {
            const double zj = kz[j];
            const int aj = ka[j];
            rank += (zj < zi || (zj == zi && aj < ai)) ? 1 : 0;
          }
        }
      }
      if (have) d.sorted[base + rank] = ai;
    }
    __syncthreads();
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
    if (l == 0) {
      for (int k = 0; k < 3; ++k) {
        const double a0 = n ? slo[k] : 0.0, a1 = n ? shi[k] : 0.0;
        d.sc_bbox[s * 6 + k] = a0;
        d.sc_bbox[s * 6 + 3 + k] = a1;
        d.sc_origin[s * 3 + k] = 0.5 * (a0 + a1);
      }
    }
  }
}

__device__ inline double gap1(double ilo, double ihi, double jlo, double jhi) {
  return fmax(0.0, fmax(jlo - ihi, ilo - jhi));
}

// Cluster-pair search, one wave per i-SC.  Candidates are walked in a fixed
// order: j-grid, x shift and column, y shift and column, j-SC in z order, z
// shift, then j-cluster.  WRITE = false counts, true writes.
template <bool WRITE>
__device__ void ph_search(const Dev& d, double rlm) {
  const double rl2 = rlm * rlm;
  const int lane = threadIdx.x & 63;
  const int ic = lane >> 3, jcq = lane & 7;  // search layout: (i-cluster, j-cluster)
  for (int s = gwave(); s < d.sc_cap; s += gwaves()) {
    if (d.sc_n[s] == 0) {
      if (!WRITE && lane == 0) d.sc_ecount[s] = 0;
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
    int count = 0;
    const int wbase = WRITE ? d.sc_estart[s] : 0;
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
              const int col = gj.col_base + cx + gj.ncx * cy;
              const int js0 = d.col_sc[col], nsc = d.col_nsc[col];
              for (int js = max(js0, s); js < js0 + nsc; ++js) {
                for (int szi = -1; szi <= 1; ++szi) {
                  const double sh[3] = {sxi * L[0], syi * L[1], szi * L[2]};
                  double g2 = 0;
                  for (int k = 0; k < 3; ++k) {
                    const double g = gap1(ilo[k], ihi[k], d.sc_bbox[js * 6 + k] + sh[k], d.sc_bbox[js * 6 + 3 + k] + sh[k]);
                    g2 += g * g;
                  }
                  if (g2 >= rl2) continue;
                  const int jcl = js * kScCl + jcq;
                  bool ok = i_ok && d.cl_n[jcl] > 0 && jcl >= icl;
                  if (ok) {
                    double c2 = 0;
                    for (int k = 0; k < 3; ++k) {
                      const double g = gap1(cilo[k], cihi[k], d.cl_bbox[jcl * 6 + k] + sh[k],
                                            d.cl_bbox[jcl * 6 + 3 + k] + sh[k]);
                      c2 += g * g;
                    }
                    ok = c2 < rl2;
                  }
                  const unsigned long long M = __ballot(ok);
                  if (M == 0) continue;
                  // lane j (0..7) gathers the i-cluster mask of j-cluster j
                  uint32_t imask = 0;
                  for (int b = 0; b < kScCl; ++b) imask |= (uint32_t)((M >> (b * 8 + (lane & 7))) & 1ull) << b;
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
    if (!WRITE && lane == 0) d.sc_ecount[s] = count;
  }
}

// Block 0 only: entry offsets per SC and the capacity check.
__device__ void ph_scan_entries(const Dev& d) {
  if (blockIdx.x != 0) return;
  const int total = block_scan_array(d.sc_ecount, d.sc_estart, d.sc_cap);
  if (threadIdx.x == 0) {
    d.ctr[CTR_ENT_NEED] = total;
    if (total > d.ent_cap) atomicOr(d.flags, 16u);
    d.ctr[CTR_NENT] = total > d.ent_cap ? 0 : total;
  }
  __syncthreads();
}

// Block 0 only: work units of at most epu entries per SC, replica ranges.
__device__ void ph_units(const Dev& d, int epu) {
  if (blockIdx.x != 0) return;
  const bool ok_all = d.ctr[CTR_NENT] == d.ctr[CTR_ENT_NEED];
  const int n = d.sc_cap;
  for (int s = threadIdx.x; s < n; s += blockDim.x) d.sc_ustart[s] = ok_all ? (d.sc_ecount[s] + epu - 1) / epu : 0;
  __syncthreads();
  const int total = block_scan_array(d.sc_ustart, d.sc_ustart, n);
  const bool fits = total <= d.unit_cap;
  if (threadIdx.x == 0) {
    d.ctr[CTR_UNIT_NEED] = total;
    d.ctr[CTR_NUNIT] = fits ? total : 0;
    if (!fits) atomicOr(d.flags, 16u);
  }
  if (fits) {
    for (int s = threadIdx.x; s < n; s += blockDim.x) {
      const int cnt = ok_all ? d.sc_ecount[s] : 0;
      if (cnt == 0) continue;
      const int u0 = d.sc_ustart[s];
      const int e0 = d.sc_estart[s];
      const int rep = d.grids[d.col_grid[d.sc_col[s]]].replica;
      for (int u = 0; u * epu < cnt; ++u) {
        const int b0 = e0 + u * epu;
        d.units[u0 + u] = make_int4(s, b0, min(e0 + cnt, b0 + epu), rep);
      }
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k <= d.n_reps; k += blockDim.x) {
    int v;
    if (!fits) v = 0;
    else if (k == d.n_reps) v = total;
    else v = d.reps[k].sc_begin < n ? d.sc_ustart[d.reps[k].sc_begin] : total;
    d.rep_ustart[k] = v;
  }
  __syncthreads();
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
  for (int e = gwave(); e < n_ent; e += gwaves()) {
    const int s = d.ent_isc[e];
    const int jc = d.ent_jc[e];
    const uint32_t info = d.ent_info[e];
    uint32_t imask = info & 0xffu;
    const int code = (int)((info >> 16) & 31u);
    const int aj = d.slot_atom[jc * kCl + jl];
    double sh[3] = {0, 0, 0};
    if (aj >= 0) {
      const ReplicaInfo& rp = d.reps[d.grids[d.atom_grid[aj]].replica];
      sh[0] = (code % 3 - 1) * rp.box[0];
      sh[1] = ((code / 3) % 3 - 1) * rp.box[1];
      sh[2] = (code / 9 - 1) * rp.box[2];
    }
    uint32_t keep = 0;
    for (int c = 0; c < kScCl; ++c) {
      bool ok = false;
      if (imask & (1u << c)) {
        const int icl = s * kScCl + c;
        const int ai = d.slot_atom[icl * kCl + il];
        if (ai >= 0 && aj >= 0 && (icl != jc || il < jl)) {
          double r2 = 0;
          for (int k = 0; k < 3; ++k) {
            const double v = d.xw[3 * aj + k] + sh[k] - d.xw[3 * ai + k];
            r2 += v * v;
          }
          ok = r2 < rl2 && !is_excluded(d, ai, aj);
        }
      }
      const unsigned long long M = __ballot(ok);
      if (M) keep |= 1u << c;
      if (lane == 0) d.ent_mask[(size_t)e * kScCl + c] = M;
    }
    if (lane == 0) {
      if (keep != imask) d.ent_info[e] = (info & ~0xffu) | keep;
      atomicAdd(&d.ctr[CTR_TILES], __popc(keep));  // 64-lane pair tiles of this list
    }
  }
}

__device__ void ph_end(const Dev& d) {
  if (gtid() == 0) {
    d.ctr[CTR_NBUILD] += 1;
    __atomic_store_n(d.rebuild, 0, __ATOMIC_RELAXED);
  }
}

// ------------------------------------------------------------ kernels

#define GATED if (!rebuild_on(d)) return
__global__ void __launch_bounds__(kBlk) k_begin(Dev d) { GATED; ph_begin(d); }
__global__ void __launch_bounds__(kBlk) k_bin(Dev d, const double* pos) { GATED; ph_bin(d, pos); }
__global__ void __launch_bounds__(kBlk) k_scan_cols(Dev d) { GATED; ph_scan_cols(d); }
__global__ void __launch_bounds__(kBlk) k_scatter(Dev d) { GATED; ph_scatter(d); }
__global__ void __launch_bounds__(kBlk) k_sort_cols(Dev d) { GATED; ph_sort_cols(d); }
__global__ void __launch_bounds__(kBlk) k_build_sc(Dev d) { GATED; ph_build_sc(d); }
__global__ void __launch_bounds__(kBlk) k_search_count(Dev d, double rlm) { GATED; ph_search<false>(d, rlm); }
__global__ void __launch_bounds__(kBlk) k_scan_entries(Dev d) { GATED; ph_scan_entries(d); }
__global__ void __launch_bounds__(kBlk) k_search_write(Dev d, double rlm) { GATED; ph_search<true>(d, rlm); }
__global__ void __launch_bounds__(kBlk) k_units(Dev d, int epu, int force) {
  if (!force) { GATED; }
  ph_units(d, epu);
}
__global__ void __launch_bounds__(kBlk) k_masks(Dev d, double rl2) { GATED; ph_masks(d, rl2); }
__global__ void __launch_bounds__(kBlk) k_end(Dev d) { GATED; ph_end(d); }
#undef GATED

static inline int clampi(long long v, int lo, int hi) { return (int)(v < lo ? lo : (v > hi ? hi : v)); }

// Grid barrier for the fused list build.  Blocks arrive on a counter and
// wait for a generation change; the wait is bounded, and a block that gives
// up raises ALCH_NB_FLAG_BARRIER_TIMEOUT and proceeds, so every wave always
// finishes.  The grid is sized on the host to fit the device at once.
__device__ inline void grid_barrier(const Dev& d, unsigned int& gen) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    unsigned int* bar = d.barrier;
    const unsigned int g = gen;
    if (atomicAdd(&bar[0], 1u) == gridDim.x - 1) {
      atomicExch(&bar[0], 0u);
      __threadfence();
      atomicAdd(&bar[1], 1u);
    } else {
      unsigned int spins = 0;
      while (__hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
        __builtin_amdgcn_s_sleep(8);
        if (++spins > (1u << 22)) {
          atomicOr(d.flags, 32u);
          break;
        }
      }
    }
    __threadfence();
    gen = g + 1;
  }
  __syncthreads();
}

// The whole list build in one launch (phases separated by grid barriers).
__global__ void __launch_bounds__(kBlk) k_list_fused(Dev d, const double* __restrict__ pos, double rlm, double rl2,
                                                     int epu) {
  if (!rebuild_on(d)) return;
  __shared__ unsigned int gen_s;
  if (threadIdx.x == 0) gen_s = __hip_atomic_load(&d.barrier[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  unsigned int gen = gen_s;
  ph_begin(d);
  grid_barrier(d, gen);
  ph_bin(d, pos);
  grid_barrier(d, gen);
  ph_scan_cols(d);
  grid_barrier(d, gen);
  ph_scatter(d);
  grid_barrier(d, gen);
  ph_sort_cols(d);
  grid_barrier(d, gen);
  ph_build_sc(d);
  grid_barrier(d, gen);
  ph_search<false>(d, rlm);
  grid_barrier(d, gen);
  ph_scan_entries(d);
  grid_barrier(d, gen);
  ph_search<true>(d, rlm);
  grid_barrier(d, gen);
  ph_units(d, epu);
  ph_masks(d, rl2);
  grid_barrier(d, gen);
  ph_end(d);
}

hipError_t launch_list_build(const Dev& d, hipStream_t st, const double* pos, double r_list, int epu,
                             int fused_blocks) {
  const double rlm = r_list * (1.0 + 1e-12) + 1e-9;  // conservative box test
  const double rl2 = rlm * rlm;  // masks keep the same margin; the export test is exact
  const dim3 B(kBlk);
  if (fused_blocks > 0) {
    hipLaunchKernelGGL(k_list_fused, dim3(fused_blocks), B, 0, st, d, pos, rlm, rl2, epu);
    return hipGetLastError();
  }
  const int g_atoms = clampi((d.n_atoms + kBlk - 1) / kBlk, 1, 512);
  const int g_cols = clampi(d.n_cols, 1, 512);
  const int g_sc = clampi((d.sc_cap + 3) / 4, 1, 512);
  const int g_ent = clampi(((long long)d.ent_cap + 3) / 4, 1, 512);
  hipLaunchKernelGGL(k_begin, dim3(clampi((d.n_cols + kBlk - 1) / kBlk, 1, 64)), B, 0, st, d);
  hipLaunchKernelGGL(k_bin, dim3(g_atoms), B, 0, st, d, pos);
  hipLaunchKernelGGL(k_scan_cols, dim3(1), B, 0, st, d);
  hipLaunchKernelGGL(k_scatter, dim3(g_atoms), B, 0, st, d);
  hipLaunchKernelGGL(k_sort_cols, dim3(g_cols), B, 0, st, d);
  hipLaunchKernelGGL(k_build_sc, dim3(g_sc), B, 0, st, d);
  hipLaunchKernelGGL(k_search_count, dim3(g_sc), B, 0, st, d, rlm);
  hipLaunchKernelGGL(k_scan_entries, dim3(1), B, 0, st, d);
  hipLaunchKernelGGL(k_search_write, dim3(g_sc), B, 0, st, d, rlm);
  hipLaunchKernelGGL(k_units, dim3(1), B, 0, st, d, epu, 0);
  hipLaunchKernelGGL(k_masks, dim3(g_ent), B, 0, st, d, rl2);
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

hipError_t launch_units(const Dev& d, hipStream_t st, int epu) {
  hipLaunchKernelGGL(k_units, dim3(1), dim3(kBlk), 0, st, d, epu, 1);
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
