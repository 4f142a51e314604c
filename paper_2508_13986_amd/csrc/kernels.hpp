// HIP kernels of the GBEES time step for gfx950 (arXiv 2508.13986).
// Included by the inst_*.hip translation units, which instantiate them per model.
//
// Per time step (Sec. 3, Fig. 1 flow: grow -> advect -> prune):
//   k_grow       directional growth (Sec. 3.3) of cells that became above the
//                threshold since the last prune; creates bricks via the hashtable;
//                keeps max_i S_i of the grown grid (Eq. 8).
//   k_grow_fix   links new bricks to their axis neighbours; finishes inserts whose
//                brick was being published by another wave.
//   k_dt         CFL time step, clamped to the stop time (Eq. 8).
//   k_flux_a     per cell: transverse fluctuations T_j and corrected states Q_l.
//   k_flux_b     per cell: DCU face fluxes of the corrected states (Eq. 7 with the
//                corner-transport terms of Algorithm 1), optional MC-limited
//                high-resolution term, conservative update, max/sum reductions.
//   k_final_step commits t, dt, max P, sum P and flips the density buffers.
// Every prune_every steps: mark (Algorithm 3), compact, rehash, relink, normalise.
//
// Gather form of Algorithm 1.  Summing the four scattered corrections of
// Algorithm 1 that land on the backward l-face of cell i gives
//   F_{i,l} = u+ Q_l(i - e_l) + u- Q_l(i),          u = f_{i - 1/2 e_l, l},
//   Q_l(k)  = P_k - sum_{j != l} dt/(2 h_j) T_j(k),
//   T_j(k)  = f+_{k-1/2e_j, j} (P_k - P_{k-e_j}) + [k+e_j in grid] f-_{k+1/2e_j, j} (P_{k+e_j} - P_k),
// where a missing cell has P = 0, and only faces with both cells present count.
// Both passes therefore touch axis neighbours only (distance <= 2 with the
// high-resolution term).
#pragma once

#include <hip/hip_runtime.h>

#include "gbees_host.hpp"

namespace gbees {

// Minimum resident waves per SIMD requested for the flux passes (caps VGPRs).
// The FP64 flux-B pass holds 4n neighbour values in flight plus its own
// corrected states; it runs fastest at two waves with no spills (measured:
// 3.8 ms per step on the Lorenz-96 6D grid, 4.6 ms at three waves with spills).
constexpr int kFluxWavesPerEU = 4;
constexpr int kFluxBWavesPerEU64 = 2, kFluxBWavesPerEU32 = 3;

// ---------------------------------------------------------------------------
// Small helpers
// ---------------------------------------------------------------------------
template <typename Real>
__device__ __forceinline__ Real rpos(Real v) { return v > Real(0) ? v : Real(0); }
template <typename Real>
__device__ __forceinline__ Real rneg(Real v) { return v < Real(0) ? v : Real(0); }

// Neighbour access inside a brick row.  For distance d along j (|d| <= side),
// lane L's neighbour sits in lane rot(L, d) of either this brick or the brick
// at sign(d) e_j: the lane whose local coordinate is (a_j + d) mod side.  Each
// lane therefore offers either its own value or the neighbour brick's value at
// its own position, and one rotate-shuffle delivers the neighbour to everyone.
template <int N>
__device__ __forceinline__ int rot_lane(int lane, int j, int d) {
  const int side = brick_side(N, j), off = brick_off(N, j);
  const int a = (lane >> off) & (side - 1);
  const int a2 = (a + d + side) & (side - 1);
  return lane + ((a2 - a) << off);
}
// Does lane `lane` serve its partner at distance d along j from its own brick?
template <int N>
__device__ __forceinline__ bool offers_own(int lane, int j, int d) {
  const int side = brick_side(N, j);
  const int a = (lane >> brick_off(N, j)) & (side - 1);
  return d > 0 ? (a >= d) : (a < side + d);
}
// The same as a lane mask.
__host__ __device__ constexpr u64 offer_own_lanes(int n, int j, int d) {
  u64 m = 0;
  for (int v = 0; v < brick_side(n, j); ++v)
    if (d > 0 ? v >= d : v < brick_side(n, j) + d) m |= lanes_at(n, j, v);
  return m;
}
// Per-lane conditions that depend only on the lane's position and on
// wave-uniform masks are formed as 64-bit lane masks with scalar
// instructions and used directly as the condition of a select.
__device__ __forceinline__ bool lane_in(u64 mask) { return __builtin_amdgcn_inverse_ballot_w64(mask); }

// Exchange with lane ^ STRIDE: DPP quad permutes for strides 1 and 2,
// ds_swizzle (bit-mask mode, within 32 lanes) for 4..16, a permute for 32.
template <int STRIDE>
__device__ __forceinline__ int xor_lane32(int v) {
  if constexpr (STRIDE == 1)
    return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
  else if constexpr (STRIDE == 2)
    return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
  else if constexpr (STRIDE < 32)
    return __builtin_amdgcn_ds_swizzle(v, (STRIDE << 10) | 0x1F);
  else
    return __shfl_xor(v, STRIDE);
}
template <int STRIDE>
__device__ __forceinline__ double xor_shfl(double v) {
  const int lo = xor_lane32<STRIDE>(__double2loint(v));
  const int hi = xor_lane32<STRIDE>(__double2hiint(v));
  return __hiloint2double(hi, lo);
}
template <int STRIDE>
__device__ __forceinline__ float xor_shfl(float v) {
  return __int_as_float(xor_lane32<STRIDE>(__float_as_int(v)));
}

// Compile-time-direction variants: J and Dd known, so the offer test is a
// constant lane mask and 2-wide dimensions use an XOR exchange.
template <int N, int J, int Dd, typename T>
__device__ __forceinline__ T nbval(T own, T other, int lane) {
  constexpr int side = brick_side(N, J), stride = brick_stride(N, J);
  if constexpr (side == 2 && (Dd == 2 || Dd == -2)) {
    return other;
  } else if constexpr (side == 2) {
    return xor_shfl<stride>(lane_in(offer_own_lanes(N, J, Dd)) ? own : other);
  } else {
    // Wider bricks test the lane's coordinate directly: selecting with the
    // constant lane mask ahead of the bpermute produced wrong neighbour
    // values for them (n = 2, 3) in the GPU parity tests.
    const T offer = offers_own<N>(lane, J, Dd) ? own : other;
    return __shfl(offer, rot_lane<N>(lane, J, Dd));
  }
}
// Lanes whose neighbour at S = +-1 along J is in the grid, given this brick's
// mask and the mask of the brick at S e_J.
template <int N, int J, int S>
__device__ __forceinline__ u64 present_lanes(u64 mown, u64 mother) {
  using D = Dir<N, J, S>;
  return (lshc<-D::sh_in>(mown) & D::in) | (lshc<-D::sh_out>(mother) & D::out);
}

// MC-limited high-resolution flux correction (LeVeque 2002, ch. 6) of one face:
// 1/2 |u| (1 - dt |u| / h) phi(theta) W.  For W, W_up of one sign,
// phi(theta) W = sign(W) min((|W| + |W_up|) / 2, 2 min(|W|, |W_up|)); else 0.
template <typename Real>
__device__ __forceinline__ Real hr_term(Real u, Real dth, Real w, Real wup) {
  const Real aw = fabs(w), awu = fabs(wup);
  const Real lim = fmin(Real(0.5) * (aw + awu), Real(2) * fmin(aw, awu));
  const Real au = fabs(u);
  const Real k = Real(0.5) * au * (Real(1) - dth * au);
  return (w * wup > Real(0)) ? k * copysign(lim, w) : Real(0);
}

// Workgroup reduction of (max, sum, count) into dpart[wg] (fixed order).
__device__ inline void wg_store3(double vmax, double vsum, double vcnt, double* dpart, uint32_t wg) {
  __shared__ double sh[3][kWavesPerWG];
  vmax = wave_max(vmax);
  vsum = wave_sum(vsum);
  vcnt = wave_sum(vcnt);
  const int w = threadIdx.x >> 6;
  if (lane_id() == 0) {
    sh[0][w] = vmax;
    sh[1][w] = vsum;
    sh[2][w] = vcnt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = sh[0][0], b = sh[1][0], c = sh[2][0];
    for (int k = 1; k < kWavesPerWG; ++k) {
      a = fmax(a, sh[0][k]);
      b = b + sh[1][k];
      c = c + sh[2][k];
    }
    dpart[wg * kPartStride + 0] = a;
    dpart[wg * kPartStride + 1] = b;
    dpart[wg * kPartStride + 2] = c;
  }
}

// Single-workgroup fixed-order reduction of G partials.
__device__ inline void reduce_partials(const double* dpart, uint32_t G, double* omax, double* osum, double* ocnt) {
  double a = 0.0, b = 0.0, c = 0.0;
  for (uint32_t i = threadIdx.x; i < G; i += blockDim.x) {
    a = fmax(a, dpart[i * kPartStride + 0]);
    b = b + dpart[i * kPartStride + 1];
    c = c + dpart[i * kPartStride + 2];
  }
  __shared__ double sh[3][kWavesPerWG];
  a = wave_max(a);
  b = wave_sum(b);
  c = wave_sum(c);
  const int w = threadIdx.x >> 6;
  if (lane_id() == 0) {
    sh[0][w] = a;
    sh[1][w] = b;
    sh[2][w] = c;
  }
  __syncthreads();
  a = sh[0][0];
  b = sh[1][0];
  c = sh[2][0];
  for (int k = 1; k < kWavesPerWG; ++k) {
    a = fmax(a, sh[0][k]);
    b = b + sh[1][k];
    c = c + sh[2][k];
  }
  *omax = a;
  *osum = b;
  *ocnt = c;
}

// ---------------------------------------------------------------------------
// Scalar kernels (one wave)
// ---------------------------------------------------------------------------
enum ScalarOp : int {
  kOpStepBegin = 0,
  kOpDt,
  kOpPruneBeginStep,
  kOpPruneBeginAlways,
  kOpPruneCommit,
  kOpSetTStop,
  kOpResetSmax,
  kOpMargBegin,
  kOpRollback,
  kOpPruneAccount
};

template <typename Real>
__device__ __forceinline__ void scalar_op(const Dev<Real>& d, int op, double arg) {
  if (threadIdx.x != 0) return;
  Scalars* sb = d.sb;
  switch (op) {
    case kOpStepBegin:
      sb->run = (sb->status == 0 && sb->t < sb->t_stop) ? 1u : 0u;
      // Steps enqueued after a failed one keep its start state for the rollback.
      if (sb->status == 0) {
        sb->nb_old = sb->nb;
        sb->smax_begin = sb->smax_bits;
      }
      sb->ndeferred = 0;
      break;
    case kOpDt: {
      if (!sb->run) break;
      if (sb->status != 0 || sb->nb > d.cap_b || sb->ndeferred > d.ndef_cap) {
        if (sb->status == 0) sb->status = kErrCapacity;
        sb->run = 0;
        break;
      }
      sb->deferred += sb->ndeferred;
      const double smax = bits_to_double(sb->smax_bits);
      const double rem = sb->t_stop - sb->t;
      double dt;
      if (d.dt_fixed > 0.0)
        dt = d.dt_fixed;
      else
        dt = (smax > 0.0) ? d.cfl / smax : rem;
      const bool last = dt >= rem;
      if (last) dt = rem;
      sb->dt = dt;
      sb->t_next = last ? sb->t_stop : sb->t + dt;
      break;
    }
    case kOpPruneBeginStep:
    case kOpPruneBeginAlways:
      sb->prun = (sb->status == 0 && (op == kOpPruneBeginAlways || sb->run)) ? 1u : 0u;
      if (sb->prun) {
        sb->smax_bits = 0ull;
        sb->nb_prev = sb->nb;
        sb->nb_new = 0;
        sb->sum_pre = sb->sum;
      }
      break;
    case kOpPruneAccount:
      // After the survivors' sum set the normaliser z = V sum: the fraction
      // of the mass present before the prune that it removed.
      if (sb->prun && sb->sum_pre > 0.0) sb->pruned += 1.0 - sb->z / (d.vol * sb->sum_pre);
      break;
    case kOpPruneCommit:
      if (!sb->prun) break;
      sb->nb = sb->nb_new;
      sb->cur ^= 1u;
      sb->prunes += 1;
      break;
    case kOpSetTStop:
      sb->t_stop = arg;
      break;
    case kOpResetSmax:
      sb->smax_bits = 0ull;
      break;
    case kOpMargBegin:
      sb->nb_new = 0;
      sb->overflow = 0;
      break;
    case kOpRollback:
      // A grow that ran out of bricks, hashtable slots or coordinate range:
      // back to the state at the start of that step (k_rollback restored the
      // masks; links are rebuilt after this).
      if (sb->status == kErrCapacity || sb->status == kErrRange) {
        sb->nb = min(sb->nb_old, d.cap_b);
        sb->smax_bits = sb->smax_begin;
        sb->status = 0;
        sb->run = 0;
        sb->prun = 0;
      }
      break;
    default:
      break;
  }
}
template <typename Real>
__global__ void k_scalar(Dev<Real> d, int op, double arg) {
  scalar_op(d, op, arg);
}

// Commit the step: reductions of the updated densities, time, buffer flip.
template <typename Real>
__device__ __forceinline__ void final_step(const Dev<Real>& d, uint32_t G) {
  Scalars* sb = d.sb;
  if (!sb->run) return;
  double a, b, c;
  reduce_partials(d.dpart, G, &a, &b, &c);
  if (threadIdx.x == 0) {
    sb->maxp = a;
    sb->sum = b;
    sb->cells = static_cast<u64>(c);
    sb->cell_updates += static_cast<u64>(c);
    sb->brick_updates += min(sb->nb, d.cap_b);
    sb->steps += 1;
    sb->dt_last = sb->dt;
    sb->t = sb->t_next;
    sb->cur ^= 1u;
  }
}
template <typename Real>
__global__ void k_final_step(Dev<Real> d, uint32_t G) {
  final_step(d, G);
}

// mode 0: sum -> normaliser z = V * sum; mode 1: max -> maxp; mode 2: max, sum, count (stats)
template <typename Real>
__global__ void k_final_reduce(Dev<Real> d, uint32_t G, int gate, int mode) {
  if (!gate_open(d, gate)) return;
  double a, b, c;
  reduce_partials(d.dpart, G, &a, &b, &c);
  if (threadIdx.x == 0) {
    Scalars* sb = d.sb;
    if (mode == 0) {
      sb->sum = b;
      sb->z = d.vol * b;
      sb->cells = static_cast<u64>(c);
    } else {
      sb->maxp = a;
      if (mode == 2) {
        sb->sum = b;
        sb->cells = static_cast<u64>(c);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Fills, hashtable build, links
// ---------------------------------------------------------------------------
template <typename Real>
__global__ void k_hash_clear(Dev<Real> d, int gate) {
  if (!gate_open(d, gate)) return;
  const uint64_t n = d.hmask + 1;
  for (uint64_t i = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x) {
    d.hkey[i] = kEmptyKey;
    d.hval[i] = kNone;
  }
}

template <typename Real>
__global__ void k_hash_insert_all(Dev<Real> d, int gate) {
  if (!gate_open(d, gate)) return;
  const uint32_t nb = nb_of(d);
  for (uint32_t b = blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += gridDim.x * blockDim.x) {
    bool won;
    const uint64_t h = hash_claim(d, d.key[b], &won);
    if (h == ~0ull) {
      set_status(d.sb, kErrCapacity);
      continue;
    }
    __hip_atomic_store(&d.hval[h], b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <int N>
__device__ __forceinline__ uint64_t neighbour_key(uint64_t key, int j, int s, bool* ok) {
  int64_t B[N];
  unpack_key<N>(key, B);
  B[j] += s;
  *ok = brick_in_range<N>(B);
  return *ok ? pack_key<N>(B) : 0ull;
}

// Link every brick in [lo, hi) to its 2n axis neighbours (thread per brick and direction);
// with `both`, also point the neighbour back (used for bricks created this step).
template <int N, typename Real>
__device__ inline void link_range(const Dev<Real>& d, uint32_t lo, uint32_t hi, bool both, Slot sl = hw_slot()) {
  const uint64_t total = static_cast<uint64_t>(hi - lo) * (2 * N);
  for (uint64_t t = sl.wg * uint64_t(blockDim.x) + threadIdx.x; t < total; t += uint64_t(sl.nwg) * blockDim.x) {
    const uint32_t b = lo + static_cast<uint32_t>(t / (2 * N));
    const int dd = static_cast<int>(t % (2 * N));
    const int j = dd >> 1, s = (dd & 1) ? 1 : -1;
    bool ok;
    const uint64_t k = neighbour_key<N>(d.key[b], j, s, &ok);
    uint32_t nbk = ok ? hash_find(d, k) : kNone;
    if (nbk != kNone && nbk >= d.cap_b) nbk = kNone;
    d.nbr[static_cast<size_t>(dd) * d.cap_b + b] = nbk;
    if (both && nbk != kNone) d.nbr[static_cast<size_t>(dd ^ 1) * d.cap_b + nbk] = b;
  }
}

template <int N, typename Real>
__global__ void k_relink_all(Dev<Real> d, int gate) {
  if (!gate_open(d, gate)) return;
  link_range<N>(d, 0u, nb_of(d), false);
}

// Undo a grow that failed (status capacity or range): bricks created since the
// step began are emptied and the older bricks get back the occupancy masks
// they had then (held in abv: flux pass A, compaction and initialisation keep
// it equal to the masks that the next step starts from).  Every done mask is
// cleared, so the next grow re-examines every source; set semantics make that
// give the same grid.  Density rows are untouched: created cells hold 0.
template <typename Real>
__global__ void k_rollback(Dev<Real> d) {
  const Scalars* sb = d.sb;
  if (sb->status != kErrCapacity && sb->status != kErrRange) return;
  const uint32_t nb_old = min(sb->nb_old, d.cap_b), nb = max(min(sb->nb, d.cap_b), nb_old);
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t b = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x; b < nb; b += stride) {
    d.mask[b] = b < nb_old ? d.abv[b] : 0ull;
    d.done[b] = 0ull;
  }
}

// ---------------------------------------------------------------------------
// Reductions over the current densities, scaling, correction
// ---------------------------------------------------------------------------
template <int N, typename Real>
__global__ __launch_bounds__(kWG) void k_reduce(Dev<Real> d, int gate) {
  if (!gate_open(d, gate)) return;
  const Real* P = cur_p(d);
  const int lane = lane_id();
  double vmax = 0.0, vsum = 0.0, vcnt = 0.0;
  const WaveRange r = wave_range(nb_of(d));
  for (uint32_t b = r.begin; b < r.end; b += r.step) {
    const u64 m = d.mask[b];
    if ((m >> lane) & 1ull) {
      const double p = static_cast<double>(P[static_cast<size_t>(b) * kLanes + lane]);
      vmax = fmax(vmax, p);
      vsum += p;
      vcnt += 1.0;
    }
  }
  wg_store3(vmax, vsum, vcnt, d.dpart, blockIdx.x);
}

// P <- P / z (z = V * sum P, Sec. 4.5 normalisation); partial max of the result.
template <int N, typename Real>
__global__ __launch_bounds__(kWG) void k_scale(Dev<Real> d, int gate) {
  if (!gate_open(d, gate)) return;
  Real* P = cur_p_mut(d);
  const double z = d.sb->z;
  const bool do_scale = z > 0.0;
  const int lane = lane_id();
  double vmax = 0.0, vsum = 0.0, vcnt = 0.0;
  const WaveRange r = wave_range(nb_of(d));
  for (uint32_t b = r.begin; b < r.end; b += r.step) {
    const size_t o = static_cast<size_t>(b) * kLanes + lane;
    double p = static_cast<double>(P[o]);
    if (do_scale) {
      p = p / z;
      P[o] = static_cast<Real>(p);
      p = static_cast<double>(static_cast<Real>(p));
    }
    if ((d.mask[b] >> lane) & 1ull) {
      vmax = fmax(vmax, p);
      vsum += p;
      vcnt += 1.0;
    }
  }
  wg_store3(vmax, vsum, vcnt, d.dpart, blockIdx.x);
}

// Bayesian correction (Eq. 4): P_i *= exp(-(y - x_i,c)^2 / (2 sigma^2)); partial max.
template <int N, typename Real>
__global__ __launch_bounds__(kWG) void k_correct(Dev<Real> d, int comp, double y, double sigma) {
  if (d.sb->status != 0) return;
  Real* P = cur_p_mut(d);
  const int lane = lane_id();
  double vmax = 0.0, vsum = 0.0, vcnt = 0.0;
  const WaveRange r = wave_range(nb_of(d));
  for (uint32_t b = r.begin; b < r.end; b += r.step) {
    int64_t B[N];
    unpack_key<N>(d.key[b], B);
    int32_t ii[N];
    double xc[N];
    cell_of<N>(d, B, lane, ii, xc);
    const size_t o = static_cast<size_t>(b) * kLanes + lane;
    double p = static_cast<double>(P[o]);
    {
#pragma clang fp contract(off)
      const double dlt = y - xc[comp];
      const double e = (dlt * dlt) / (2.0 * sigma * sigma);
      p = p * exp(-e);
    }
    P[o] = static_cast<Real>(p);
    if ((d.mask[b] >> lane) & 1ull) {
      vmax = fmax(vmax, static_cast<double>(static_cast<Real>(p)));
      vsum += p;
      vcnt += 1.0;
    }
  }
  wg_store3(vmax, vsum, vcnt, d.dpart, blockIdx.x);
}

// S over every cell of the grid (after initialisation).
template <int N, int MODEL, typename Real>
__global__ __launch_bounds__(kWG) void k_smax_all(Dev<Real> d) {
  const int lane = lane_id();
  double smax = 0.0;
  const WaveRange r = wave_range(nb_of(d));
  for (uint32_t b = r.begin; b < r.end; b += r.step) {
    const u64 m = d.mask[b];
    if ((m >> lane) & 1ull) {
      int64_t B[N];
      unpack_key<N>(d.key[b], B);
      int32_t ii[N];
      double xc[N];
      cell_of<N>(d, B, lane, ii, xc);
      smax = fmax(smax, cell_speed<MODEL, N>(d, xc, ii));
    }
  }
  smax = wave_max(smax);
  if (lane == 0 && smax > 0.0) atomicMax(&d.sb->smax_bits, double_to_bits(smax));
}

// ---------------------------------------------------------------------------
// Initial condition (ellipsoid of the Gaussian)
// ---------------------------------------------------------------------------
template <int N, typename Real>
__device__ __forceinline__ void box_brick(const Dev<Real>& d, uint64_t lin, int64_t* B) {
#pragma unroll
  for (int j = 0; j < N; ++j) {
    B[j] = d.box_lo[j] + static_cast<int64_t>(lin % static_cast<uint64_t>(d.box_n[j]));
    lin /= static_cast<uint64_t>(d.box_n[j]);
  }
}

// q(i) = y' S^-1 y with y = i h, in a fixed operation order.
template <int N, typename Real>
__device__ __forceinline__ double quad_form(const Dev<Real>& d, const int32_t* ii) {
#pragma clang fp contract(off)
  double y[N];
#pragma unroll
  for (int j = 0; j < N; ++j) y[j] = static_cast<double>(ii[j]) * d.h[j];
  double q = 0.0;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    double row = 0.0;
#pragma unroll
    for (int k = 0; k < N; ++k) row = row + d.sinv[j * N + k] * y[k];
    q = q + y[j] * row;
  }
  return q;
}

template <int N, typename Real>
__global__ __launch_bounds__(kWG) void k_init_count(Dev<Real> d) {
  uint64_t lo, hi;
  wg_chunk(d.box_count, lo, hi);
  const int lane = lane_id(), w = threadIdx.x >> 6;
  uint32_t cnt = 0;
  for (uint64_t i = lo + w; i < hi; i += kWavesPerWG) {
    int64_t B[N];
    box_brick<N>(d, i, B);
    int32_t ii[N];
    double xc[N];
    cell_of<N>(d, B, lane, ii, xc);
    if (ballot(quad_form<N>(d, ii) <= d.bound) != 0ull) ++cnt;
  }
  __shared__ uint32_t sh[kWavesPerWG];
  if (lane == 0) sh[w] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t s = 0;
    for (int k = 0; k < kWavesPerWG; ++k) s += sh[k];
    d.part[blockIdx.x] = s;
  }
}

template <int N, typename Real>
__global__ __launch_bounds__(kWG) void k_init_write(Dev<Real> d) {
  uint64_t lo, hi;
  wg_chunk(d.box_count, lo, hi);
  const int lane = lane_id(), w = threadIdx.x >> 6;
  uint32_t base = d.part[blockIdx.x];
  __shared__ uint32_t sh[kWavesPerWG];
  for (uint64_t r0 = lo; r0 < hi; r0 += kWavesPerWG) {
    const uint64_t i = r0 + w;
    int64_t B[N];
    int32_t ii[N];
    double xc[N];
    double q = 0.0;
    u64 m = 0;
    if (i < hi) {
      box_brick<N>(d, i, B);
      cell_of<N>(d, B, lane, ii, xc);
      q = quad_form<N>(d, ii);
      m = ballot(q <= d.bound);
    }
    if (lane == 0) sh[w] = (m != 0ull) ? 1u : 0u;
    __syncthreads();
    uint32_t before = 0, total = 0;
    for (int k = 0; k < kWavesPerWG; ++k) {
      before += (k < w) ? sh[k] : 0u;
      total += sh[k];
    }
    if (m != 0ull) {
      const uint32_t dst = base + before;
      if (dst < d.cap_b) {
        if (lane == 0) {
          d.key[dst] = pack_key<N>(B);
          d.mask[dst] = m;
          d.abv[dst] = m;
        }
        const bool in = (m >> lane) & 1ull;
        Real* P = d.P0;
        P[static_cast<size_t>(dst) * kLanes + lane] = in ? static_cast<Real>(exp(-q / 2.0)) : Real(0);
      }
    }
    base += total;
    __syncthreads();
  }
}

// Exclusive scan of part[0, G) in place; the total goes to part[G] and *total.
static __global__ void k_scan(uint32_t* part, uint32_t G, Scalars* sb, int gate, uint32_t* total, uint32_t cap) {
  if (gate == kGatePrune && !sb->prun) return;
  __shared__ uint32_t sh[kWG];
  const uint32_t per = (G + kWG - 1) / kWG;
  const uint32_t lo = threadIdx.x * per, hi = min(G, lo + per);
  uint32_t s = 0;
  for (uint32_t i = lo; i < hi; ++i) s += part[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t acc = 0;
    for (int k = 0; k < kWG; ++k) {
      const uint32_t v = sh[k];
      sh[k] = acc;
      acc += v;
    }
    part[G] = acc;
    if (acc > cap) {
      atomicCAS(&sb->status, 0, static_cast<int32_t>(kErrCapacity));
      acc = cap;
    }
    *total = acc;
  }
  __syncthreads();
  uint32_t acc = sh[threadIdx.x];
  for (uint32_t i = lo; i < hi; ++i) {
    const uint32_t v = part[i];
    part[i] = acc;
    acc += v;
  }
}

// ---------------------------------------------------------------------------
// Grow (Sec. 3.3, Algorithm 2 semantics as set union over the pre-grow grid)
// ---------------------------------------------------------------------------
// S of this lane's cell in the brick with coordinates TB if the lane is one of
// `created`, else 0.
template <int N, int MODEL, typename Real>
__device__ __forceinline__ double created_speed(const Dev<Real>& d, const int64_t* TB, u64 created, int lane) {
  double s = 0.0;
  if ((created >> lane) & 1ull) {
    int32_t ii[N];
    double xc[N];
    cell_of<N>(d, TB, lane, ii, xc);
    s = cell_speed<MODEL, N>(d, xc, ii);
  }
  return s;
}

// Adds the cells `bits` to the brick with coordinates TB (index tb, or kNone if
// unknown).  Returns the largest S of the cells this call created (wave-uniform).
template <int N, int MODEL, typename Real>
__device__ __forceinline__ double add_cells(const Dev<Real>& d, const int64_t* TB, uint32_t tb, u64 bits, int lane,
                                            u64* created_count) {
  if (tb == kNone) {
    if (!brick_in_range<N>(TB)) {
      if (lane == 0) set_status(d.sb, kErrRange);
      return 0.0;
    }
    const uint64_t key = pack_key<N>(TB);
    uint64_t hs = 0;
    int won = 0;
    if (lane == 0) {
      bool w;
      hs = hash_claim(d, key, &w);
      won = w ? 1 : 0;
    }
    hs = __shfl(hs, 0);
    won = __shfl(won, 0);
    if (hs == ~0ull) {
      if (lane == 0) set_status(d.sb, kErrCapacity);
      return 0.0;
    }
    if (won) {
      uint32_t slot = 0;
      if (lane == 0) {
        slot = atomicAdd(&d.sb->nb, 1u);
        if (slot < d.cap_b) {
          d.key[slot] = key;
          __hip_atomic_store(&d.hval[hs], slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
          set_status(d.sb, kErrCapacity);
        }
      }
      slot = __shfl(slot, 0);
      if (slot >= d.cap_b) return 0.0;
      tb = slot;
    } else {
      uint32_t v = 0;
      if (lane == 0) v = __hip_atomic_load(&d.hval[hs], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      v = __shfl(v, 0);
      if (v == kNone) {
        // Claimed by another wave that has not published the brick index yet.
        if (lane == 0) {
          const uint32_t k = atomicAdd(&d.sb->ndeferred, 1u);
          if (k < d.ndef_cap) {
            d.defer[2 * static_cast<size_t>(k)] = hs;
            d.defer[2 * static_cast<size_t>(k) + 1] = bits;
          }
        }
        return 0.0;
      }
      tb = v;
    }
  }
  // A stale (smaller) mask only costs an extra atomicOr.
  const u64 cur = d.mask[tb];
  if ((bits & ~cur) == 0ull) return 0.0;
  u64 old = 0;
  if (lane == 0) old = atomicOr(&d.mask[tb], bits);
  old = __shfl(old, 0);
  const u64 created = bits & ~old;
  if (created == 0ull) return 0.0;
  *created_count += static_cast<u64>(__popcll(created));
  return wave_max(created_speed<N, MODEL>(d, TB, created, lane));
}

template <typename Real>
__device__ __forceinline__ uint32_t nbr_of(const Dev<Real>& d, uint32_t b, int j, int s) {
  return b == kNone ? kNone : d.nbr[static_cast<size_t>(2 * j + (s > 0 ? 1 : 0)) * d.cap_b + b];
}

// Per-brick metadata of the flux passes, gathered into one VGPR so that the
// next brick's links, mask and key can be fetched while the current brick is
// computed: lane 2j + s holds the link to the brick at (s ? +1 : -1) e_j, lanes
// 2n, 2n + 1 the occupancy mask and lanes 2n + 2, 2n + 3 the key (low word
// first).  Each lane reads one 32-bit word at base + (b << shift), with its
// base and shift fixed for the whole launch (MetaLane); b == kNone loads
// nothing.
struct MetaLane {
  const char* base;
  uint32_t shift;
};
template <int N, typename Real>
__device__ __forceinline__ MetaLane meta_lane(const Dev<Real>& d, int lane) {
  if (lane < 2 * N) return {reinterpret_cast<const char*>(d.nbr + static_cast<size_t>(lane) * d.cap_b), 2};
  if (lane < 2 * N + 2) return {reinterpret_cast<const char*>(d.mask) + 4 * (lane - 2 * N), 3};
  return {reinterpret_cast<const char*>(d.key) + 4 * (lane - 2 * N - 2), 3};
}
template <int N>
__device__ __forceinline__ uint32_t meta_fetch(MetaLane ml, uint32_t b) {
  constexpr u64 kMetaLanes = (1ull << (2 * N + 4)) - 1;
  uint32_t v = 0;
  if (b != kNone && lane_in(kMetaLanes)) v = *reinterpret_cast<const uint32_t*>(ml.base + (static_cast<size_t>(b) << ml.shift));
  return v;
}
template <int N>
struct BrickMeta {
  uint32_t bm[N], bp[N];
  u64 mask, key;
};
template <int N>
__device__ __forceinline__ BrickMeta<N> meta_unpack(uint32_t v) {
  BrickMeta<N> r;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    r.bm[j] = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v), 2 * j));
    r.bp[j] = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v), 2 * j + 1));
  }
  auto word = [&](int k) { return static_cast<u64>(static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v), k))); };
  r.mask = word(2 * N) | (word(2 * N + 1) << 32);
  r.key = word(2 * N + 2) | (word(2 * N + 3) << 32);
  return r;
}

// Targets of one brick: 0 = the brick itself, 1 + 2j + si = the axis neighbour
// at s e_j (si = s > 0), then for each pair j < l and signs (s, r) the edge
// neighbour at s e_j + r e_l.  Count: 1 + 2n + 4 n(n-1)/2.
__host__ __device__ constexpr int n_targets(int n) { return 1 + 2 * n + 2 * n * (n - 1); }

template <int N>
__device__ __forceinline__ int target_kind(int k, int* j, int* s, int* l, int* r) {
  if (k == 0) return 0;
  if (k < 1 + 2 * N) {
    *j = (k - 1) >> 1;
    *s = ((k - 1) & 1) ? 1 : -1;
    return 1;
  }
  int q = k - 1 - 2 * N;
  int p = q >> 2;
  *s = ((q >> 1) & 1) ? 1 : -1;
  *r = (q & 1) ? 1 : -1;
  int jj = 0;
  while (p >= N - 1 - jj) {
    p -= N - 1 - jj;
    ++jj;
  }
  *j = jj;
  *l = jj + 1 + p;
  return 2;
}

// Axis links of brick b spread over the wave: lane 1 + 2j + si holds the index
// of the brick at (si ? +1 : -1) e_j, every other lane kNone.
template <int N, typename Real>
__device__ __forceinline__ uint32_t axis_links(const Dev<Real>& d, uint32_t b, int lane) {
  return (lane >= 1 && lane < 1 + 2 * N) ? d.nbr[static_cast<size_t>(lane - 1) * d.cap_b + b] : kNone;
}

// Index of target k of brick b through the link table, kNone if the links do
// not reach it (and for lanes whose `want` is false); axl holds b's axis links
// (axis_links).  An edge target s e_j + r e_l is reached via the brick at s e_j,
// else via the one at r e_l.  Axis targets and the first hop of edge targets
// come from the axis lanes, so an edge target costs one link load, two when its
// first route is missing.  Every lane of the wave must take part (the hops are
// lane shuffles).
template <int N, typename Real>
__device__ __forceinline__ uint32_t resolve_target(const Dev<Real>& d, uint32_t b, int k, uint32_t axl, bool want) {
  int j = 0, s = 0, l = 0, r = 0;
  const int kind = k < n_targets(N) ? target_kind<N>(k, &j, &s, &l, &r) : -1;
  const uint32_t h1 = static_cast<uint32_t>(__shfl(static_cast<int>(axl), kind >= 1 ? 1 + 2 * j + (s > 0 ? 1 : 0) : 0));
  const uint32_t h2 = static_cast<uint32_t>(__shfl(static_cast<int>(axl), kind == 2 ? 1 + 2 * l + (r > 0 ? 1 : 0) : 0));
  if (!want || kind < 0) return kNone;
  if (kind == 0) return b;
  if (kind == 1) return h1;
  uint32_t t = nbr_of(d, h1, l, r);
  if (t == kNone) t = nbr_of(d, h2, j, s);
  return t;
}

// A wave-uniform value moved to scalar registers.
__device__ __forceinline__ double uniform(double v) {
  const u64 b = double_to_bits(v);
  const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(b));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(b >> 32));
  return bits_to_double((static_cast<u64>(hi) << 32) | lo);
}
__device__ __forceinline__ float uniform(float v) {
  return __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(v)));
}

// Orders this wave's LDS writes before its lanes read what other lanes wrote.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ u64 readlane64(u64 v, int k) {
  const uint32_t lo = __builtin_amdgcn_readlane(static_cast<uint32_t>(v), k);
  const uint32_t hi = __builtin_amdgcn_readlane(static_cast<uint32_t>(v >> 32), k);
  return (static_cast<u64>(hi) << 32) | lo;
}

// Word w of target k, held by lane k (k < 64) or lane k - 64 of the second set.
__device__ __forceinline__ u64 target_word(u64 w0, u64 w1, int k) { return k < 64 ? readlane64(w0, k) : readlane64(w1, k - 64); }
__device__ __forceinline__ uint32_t target_index(uint32_t t0, uint32_t t1, int k) {
  return k < 64 ? __builtin_amdgcn_readlane(t0, k) : __builtin_amdgcn_readlane(t1, k - 64);
}

// Bricks whose density rows are fetched together by the grow scan.
constexpr int kGrowBatch = 8;

// Brick coordinates of target k of the brick with coordinates B.
template <int N>
__device__ __forceinline__ void target_coords(const int64_t* B, int k, int64_t* TB) {
  int j = 0, s = 0, l = 0, r = 0;
  const int kind = target_kind<N>(k, &j, &s, &l, &r);
  // Static indexes only: a runtime index would put TB in scratch memory.
#pragma unroll
  for (int q = 0; q < N; ++q) TB[q] = B[q] + (kind >= 1 && q == j ? s : 0) + (kind == 2 && q == l ? r : 0);
}

// The moves of grow: 2n axis moves (s e_j) and, per pair j < l, four edge
// moves (s e_j + r e_l).  A move carries a source set (the new sources whose
// downwind directions include it) to candidate cells in up to four target
// bricks, one per quadrant of the brick: lanes that stay inside along both
// axes (the brick itself), that leave along j only (the axis neighbour at
// s e_j), along l only (the one at r e_l), or along both (the edge
// neighbour).  Each quadrant is a lane mask and a lane shift, fixed by the
// brick shape; the table below holds them per move so that every lane of a
// wave can apply one move.
template <int N>
struct MoveTable {
  static constexpr int kMoves = 2 * N + 2 * N * (N - 1);
  u64 q[4][kMoves];       // quadrant lane masks
  uint32_t sh[4][kMoves];  // left shift | right shift << 8 (one of them 0)
  uint32_t tg[kMoves];     // target of quadrant i in byte i (0xFF: none)
  uint32_t src[kMoves];    // source set index a | b << 8 (b = 0xFF: all lanes)
};
// The table of a brick shape, built at compile time: entry m < 2n is the axis
// move s e_j (j = m / 2, s = +1 for odd m), then four edge moves per pair
// j < l in pair order (s, r = -1, -1; -1, +1; +1, -1; +1, +1).  Quadrant 0
// keeps the lanes that stay inside along both axes, 1 those that leave along
// j only, 2 along l only, 3 along both; a shift is coded as left | right << 8.
template <int N>
constexpr MoveTable<N> make_moves() {
  MoveTable<N> t{};
  auto out = [](int j, int s) { return s > 0 ? lanes_at(N, j, brick_side(N, j) - 1) : lanes_at(N, j, 0); };
  auto sh_in = [](int j, int s) { return s * brick_stride(N, j); };
  auto sh_out = [](int j, int s) { return -s * (brick_side(N, j) - 1) * brick_stride(N, j); };
  auto code = [](int k) { return k >= 0 ? static_cast<uint32_t>(k) : static_cast<uint32_t>(-k) << 8; };
  int m = 0;
  for (int j = 0; j < N; ++j)
    for (int si = 0; si < 2; ++si, ++m) {
      const int s = si ? 1 : -1;
      t.q[0][m] = ~out(j, s);
      t.q[1][m] = out(j, s);
      t.sh[0][m] = code(sh_in(j, s));
      t.sh[1][m] = code(sh_out(j, s));
      t.tg[m] = static_cast<uint32_t>(1 + 2 * j + si) << 8 | 0xFFu << 16 | 0xFFu << 24;
      t.src[m] = static_cast<uint32_t>(2 * j + si) | 0xFFu << 8;
    }
  for (int p = 0; p < N * (N - 1) / 2; ++p) {
    const int j = pair_j(N, p), l = pair_l(N, p);
    for (int c = 0; c < 4; ++c, ++m) {
      const int si = c >> 1, ri = c & 1, s = si ? 1 : -1, r = ri ? 1 : -1;
      const u64 oj = out(j, s), ol = out(l, r);
      t.q[0][m] = ~oj & ~ol;
      t.q[1][m] = oj & ~ol;
      t.q[2][m] = ~oj & ol;
      t.q[3][m] = oj & ol;
      t.sh[0][m] = code(sh_in(j, s) + sh_in(l, r));
      t.sh[1][m] = code(sh_out(j, s) + sh_in(l, r));
      t.sh[2][m] = code(sh_in(j, s) + sh_out(l, r));
      t.sh[3][m] = code(sh_out(j, s) + sh_out(l, r));
      t.tg[m] = static_cast<uint32_t>(1 + 2 * j + si) << 8 | static_cast<uint32_t>(1 + 2 * l + ri) << 16 |
                static_cast<uint32_t>(1 + 2 * N + 4 * p + 2 * si + ri) << 24;
      t.src[m] = static_cast<uint32_t>(2 * j + si) | static_cast<uint32_t>(2 * l + ri) << 8;
    }
  }
  return t;
}
template <int N>
__device__ const MoveTable<N> kMoveTable = make_moves<N>();
// Copies the table into a workgroup's LDS, a word per thread at a time
// (callers synchronise afterwards).
template <int N>
__device__ __forceinline__ void fill_moves(MoveTable<N>& t) {
  static_assert(sizeof(MoveTable<N>) % 4 == 0, "whole words");
  const uint32_t* src = reinterpret_cast<const uint32_t*>(&kMoveTable<N>);
  uint32_t* dst = reinterpret_cast<uint32_t*>(&t);
  for (uint32_t i = threadIdx.x; i < sizeof(MoveTable<N>) / 4; i += blockDim.x) dst[i] = src[i];
}

// Grow in two phases per wave.  Phase one takes the bricks with new sources
// one at a time: it marks their sources done and turns the sources' downwind
// directions into candidate cells per target brick (the brick itself, its 2n
// axis neighbours and its edge neighbours), which it appends to a list in LDS.
// Phase two runs whenever the list holds a wave's worth of entries: each lane
// resolves one (brick, target) entry through the links, reads the target's
// mask and adds the missing cells with one atomic, so the dependent round
// trips of many bricks are in flight together instead of one brick after
// another.  Targets the links do not reach go through the hashtable, one at a
// time.  The order in which targets receive their cells does not matter: the
// grown set is the union over all sources of the pre-grow grid.
//
// Four waves per SIMD (measured faster than five or more, which spill).
template <int N, int MODEL, typename Real>
__device__ __forceinline__ void grow_body(const Dev<Real>& d, Slot sl) {
  Scalars* sb = d.sb;
  if (!sb->run) return;
  const uint32_t nb_old = sb->nb_old;
  const Real* P = cur_p(d);
  const bool thr0 = !(d.thresh_rel > 0.0);
  // p* in scalar registers (a vector copy was spilled and reloaded per brick).
  const Real pstar = uniform(static_cast<Real>(d.thresh_rel * sb->maxp));
  const int lane = lane_id();
  constexpr int NT = n_targets(N);
  constexpr int kEnt = kLanes + NT;  // one resolution round plus one brick's targets
  __shared__ u64 tbl_all[kWavesPerWG][128];
  __shared__ u64 work_all[kWavesPerWG][5 * kGrowBatch];
  __shared__ u64 ebits_all[kWavesPerWG][kEnt];
  __shared__ u64 ekey_all[kWavesPerWG][kEnt];
  __shared__ uint32_t eb_all[kWavesPerWG][kEnt];
  __shared__ uint32_t ek_all[kWavesPerWG][kEnt];
  __shared__ u64 ud_all[kWavesPerWG][2 * N];
  __shared__ MoveTable<N> mt;
  fill_moves<N>(mt);
  __syncthreads();
  const int wv = threadIdx.x >> 6;
  u64* ud = ud_all[wv];
  u64* tbl = tbl_all[wv];
  u64* work = work_all[wv];
  u64* ebits = ebits_all[wv];
  u64* ekey = ekey_all[wv];
  uint32_t* eb = eb_all[wv];
  uint32_t* ek = ek_all[wv];
  uint32_t nent = 0;  // entries in the list (wave-uniform)
  double smax = 0.0;
  u64 nscan = 0, ncreated = 0;

  // Phase two over the first `cnt` (<= 64) entries.
  auto resolve = [&](uint32_t cnt) {
    const bool live = static_cast<uint32_t>(lane) < cnt;
    const u64 bits = live ? ebits[lane] : 0ull;
    const uint32_t b = live ? eb[lane] : kNone;
    const int k = live ? static_cast<int>(ek[lane]) : 0;
    uint32_t t = kNone;
    if (live) {
      int j = 0, s = 0, l = 0, r = 0;
      const int kind = target_kind<N>(k, &j, &s, &l, &r);
      if (kind == 0) {
        t = b;
      } else {
        // An edge target s e_j + r e_l is reached via the brick at s e_j, else
        // via the one at r e_l.
        const uint32_t h1 = nbr_of(d, b, j, s);
        if (kind == 1) {
          t = h1;
        } else {
          t = nbr_of(d, h1, l, r);
          if (t == kNone) t = nbr_of(d, nbr_of(d, b, l, r), j, s);
        }
      }
    }
    // Most targets already hold their candidate cells: a plain load of the
    // target's mask settles those, and only cells still missing take the
    // (device-scope) atomic.  A stale mask only costs an atomic.
    const u64 need = (live && t != kNone) ? bits & ~d.mask[t] : 0ull;
    u64 made = 0ull;
    if (need != 0ull) made = need & ~atomicOr(&d.mask[t], need);
    u64 made_t = ballot(made != 0ull);
    u64 hash_t = ballot(live && t == kNone);
    while (made_t != 0ull) {
      const int kl = __builtin_ctzll(made_t);
      made_t &= made_t - 1ull;
      const u64 mk = readlane64(made, kl);
      int64_t B[N], TB[N];
      unpack_key<N>(readlane64(ekey[lane], kl), B);
      target_coords<N>(B, __builtin_amdgcn_readlane(k, kl), TB);
      ncreated += static_cast<u64>(__popcll(mk));
      smax = fmax(smax, created_speed<N, MODEL>(d, TB, mk, lane));
    }
    while (hash_t != 0ull) {
      const int kl = __builtin_ctzll(hash_t);
      hash_t &= hash_t - 1ull;
      const u64 bk = readlane64(bits, kl);
      int64_t B[N], TB[N];
      unpack_key<N>(readlane64(ekey[lane], kl), B);
      target_coords<N>(B, __builtin_amdgcn_readlane(k, kl), TB);
      smax = fmax(smax, add_cells<N, MODEL>(d, TB, kNone, bk, lane, &ncreated));
    }
  };

  // Phase one for brick b with key `key` (m: occupancy, dn_new: the done mask
  // after this step, todo: the new sources).
  auto grow_brick = [&](uint32_t b, u64 key, u64 m, u64 dn_new, u64 todo) {
    if (lane == 0) {
      d.done[b] = dn_new;
      ++nscan;
    }
    int64_t B[N];
    unpack_key<N>(key, B);
    int32_t ii[N];
    double xc[N];
    cell_of<N>(d, B, lane, ii, xc);
    const bool t = (todo >> lane) & 1ull;
    u64 U[N], D[N];  // todo lanes with a downwind +e_j / -e_j neighbour
#pragma unroll
    for (int j = 0; j < N; ++j) {
      bool up = t, dw = t;
      if (d.grow_mode == 0) {
        up = t && face_vel_fwd<MODEL, N>(d, xc, ii, j) > 0.0;
        dw = t && face_vel<MODEL, N>(d, xc, ii, j) < 0.0;
      }
      U[j] = ballot(up);
      D[j] = ballot(dw);
    }
    // Candidate cells of every target brick into the wave's table (entry 0 the
    // brick itself, 1 + 2j + si the axis neighbours, then the edge
    // neighbours): lane i applies move i (and i + 64), OR-ing its quadrants
    // into the targets they reach; an edge target has only its own move.
    tbl[lane] = 0ull;
    tbl[lane + 64] = 0ull;
    if (lane == 0) {
#pragma unroll
      for (int j = 0; j < N; ++j) {
        ud[2 * j] = D[j];
        ud[2 * j + 1] = U[j];
      }
    }
    wave_lds_sync();
    constexpr int kMoves = MoveTable<N>::kMoves;
#pragma unroll
    for (int rnd = 0; rnd * kLanes < kMoves; ++rnd) {
      const int mv = lane + rnd * kLanes;
      if (mv < kMoves) {
        const uint32_t sc = mt.src[mv];
        const u64 sa = ud[sc & 0xFFu];
        const u64 both = (sc >> 8) == 0xFFu ? sa : sa & ud[sc >> 8];
        if (both != 0ull) {
          const uint32_t tg = mt.tg[mv];
#pragma unroll
          for (int qd = 0; qd < 4; ++qd) {
            const uint32_t sh = mt.sh[qd][mv];
            const u64 v = ((both & mt.q[qd][mv]) << (sh & 0xFFu)) >> (sh >> 8);
            const uint32_t k = (tg >> (8 * qd)) & 0xFFu;
            if (v != 0ull && k != 0xFFu) {
              if (qd == 3)
                tbl[k] = v;
              else
                atomicOr(reinterpret_cast<unsigned long long*>(&tbl[k]), static_cast<unsigned long long>(v));
            }
          }
        }
      }
    }
    wave_lds_sync();
    // Append the targets that received candidates (the brick itself: the
    // cells it does not hold yet).
    const u64 bits0 = lane == 0 ? tbl[0] & ~m : tbl[lane];
    const u64 bits1 = lane + 64 < NT ? tbl[lane + 64] : 0ull;
    const u64 nz0 = ballot(bits0 != 0ull), nz1 = ballot(bits1 != 0ull);
    const u64 below = (1ull << lane) - 1ull;
    if (bits0 != 0ull) {
      const uint32_t at = nent + static_cast<uint32_t>(__popcll(nz0 & below));
      ebits[at] = bits0;
      ekey[at] = key;
      eb[at] = b;
      ek[at] = static_cast<uint32_t>(lane);
    }
    if (bits1 != 0ull) {
      const uint32_t at = nent + static_cast<uint32_t>(__popcll(nz0) + __popcll(nz1 & below));
      ebits[at] = bits1;
      ekey[at] = key;
      eb[at] = b;
      ek[at] = static_cast<uint32_t>(lane + 64);
    }
    nent += static_cast<uint32_t>(__popcll(nz0) + __popcll(nz1));
    wave_lds_sync();
    while (nent >= static_cast<uint32_t>(kLanes)) {
      resolve(kLanes);
      // Move the remaining entries (fewer than NT) to the front: read them
      // all before writing any (the ranges overlap for NT > 64).
      const uint32_t rest = nent - kLanes;
      const uint32_t i0 = static_cast<uint32_t>(lane), i1 = static_cast<uint32_t>(lane) + kLanes;
      const bool m0 = i0 < rest, m1 = i1 < rest;
      u64 vb0 = 0ull, vk0 = 0ull, vb1 = 0ull, vk1 = 0ull;
      uint32_t b0 = 0, k0 = 0, b1 = 0, k1 = 0;
      if (m0) { vb0 = ebits[kLanes + i0]; vk0 = ekey[kLanes + i0]; b0 = eb[kLanes + i0]; k0 = ek[kLanes + i0]; }
      if (m1) { vb1 = ebits[kLanes + i1]; vk1 = ekey[kLanes + i1]; b1 = eb[kLanes + i1]; k1 = ek[kLanes + i1]; }
      wave_lds_sync();
      if (m0) { ebits[i0] = vb0; ekey[i0] = vk0; eb[i0] = b0; ek[i0] = k0; }
      if (m1) { ebits[i1] = vb1; ekey[i1] = vk1; eb[i1] = b1; ek[i1] = k1; }
      wave_lds_sync();
      nent = rest;
    }
  };

  // The scan takes runs of up to kRunMax bricks: lane i reads the occupancy and
  // done masks of brick r + i, and only bricks holding a cell that has not yet been a
  // source are candidates.  Their density rows are fetched kGrowBatch at a time
  // so the round trips overlap; bricks with new sources are queued in LDS and
  // grown one by one.  A stale mask is harmless: cells added concurrently hold
  // P = 0 and are no sources.
  const RunRange rr = wave_runs(nb_old, sl);
  for (uint32_t r = rr.begin; r < rr.end; r += rr.step) {
    const uint32_t bl = r + static_cast<uint32_t>(lane);
    u64 ml = 0ull, dl = 0ull, kyl = 0ull;
    if (static_cast<uint32_t>(lane) < rr.len && bl < rr.end) {
      ml = d.mask[bl];
      dl = d.done[bl];
      kyl = d.key[bl];
    }
    u64 cand = ballot((ml & ~dl) != 0ull);
    while (cand != 0ull) {
      uint32_t bk[kGrowBatch];
      u64 mk[kGrowBatch], dk[kGrowBatch], kk[kGrowBatch];
      Real pk[kGrowBatch];
#pragma unroll
      for (int k = 0; k < kGrowBatch; ++k) {
        bk[k] = kNone;
        mk[k] = dk[k] = kk[k] = 0ull;
        pk[k] = Real(0);
        if (cand != 0ull) {
          const int kl = __builtin_ctzll(cand);
          cand &= cand - 1ull;
          bk[k] = r + static_cast<uint32_t>(kl);
          mk[k] = readlane64(ml, kl);
          dk[k] = readlane64(dl, kl);
          kk[k] = readlane64(kyl, kl);
          pk[k] = P[static_cast<size_t>(bk[k]) * kLanes + lane];
        }
      }
      int nwork = 0;
#pragma unroll
      for (int k = 0; k < kGrowBatch; ++k) {
        if (bk[k] == kNone) break;
        const bool src = ((mk[k] >> lane) & 1ull) && (thr0 ? (pk[k] != Real(0)) : (pk[k] >= pstar));
        const u64 S = ballot(src);
        const u64 todo = S & ~dk[k];
        if (todo != 0ull) {
          if (lane == 0) {
            work[5 * nwork] = bk[k];
            work[5 * nwork + 1] = mk[k];
            work[5 * nwork + 2] = dk[k] | S;
            work[5 * nwork + 3] = todo;
            work[5 * nwork + 4] = kk[k];
          }
          ++nwork;
        }
      }
      if (nwork == 0) continue;
      wave_lds_sync();
      for (int w = 0; w < nwork; ++w) {
        const uint32_t b = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<uint32_t>(work[5 * w])));
        const u64 m = readlane64(work[5 * w + 1], 0);
        const u64 dn_new = readlane64(work[5 * w + 2], 0);
        const u64 todo = readlane64(work[5 * w + 3], 0);
        const u64 key = readlane64(work[5 * w + 4], 0);
        grow_brick(b, key, m, dn_new, todo);
      }
    }
  }
  if (nent > 0) resolve(nent);
  smax = wave_max(smax);
  if (lane == 0 && smax > 0.0) atomicMax(&sb->smax_bits, double_to_bits(smax));
  if (lane == 0 && nscan > 0) atomicAdd(&sb->grow_bricks, nscan);
  if (lane == 0 && ncreated > 0) atomicAdd(&sb->inserted, ncreated);
}
template <int N, int MODEL, typename Real>
__global__ __launch_bounds__(kWG, 4) void k_grow(Dev<Real> d) {
  grow_body<N, MODEL, Real>(d, hw_slot());
}

// Link the bricks created this step and finish inserts that found their brick unpublished.
template <int N, int MODEL, typename Real>
__device__ __forceinline__ void grow_fix_body(const Dev<Real>& d, Slot sl) {
  Scalars* sb = d.sb;
  if (!sb->run || sb->status != 0) return;
  const uint32_t nb = min(sb->nb, d.cap_b), nb_old = sb->nb_old;
  if (nb > nb_old) link_range<N>(d, nb_old, nb, true, sl);
  const uint32_t ndef = min(sb->ndeferred, d.ndef_cap);
  const int lane = lane_id();
  double smax = 0.0;
  u64 ncreated = 0;
  const uint32_t wid = sl.wg * kWavesPerWG + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t nw = sl.nwg * kWavesPerWG;
  for (uint32_t k = wid; k < ndef; k += nw) {
    const uint64_t hs = d.defer[2 * static_cast<size_t>(k)];
    const u64 bits = d.defer[2 * static_cast<size_t>(k) + 1];
    const uint32_t tb = __hip_atomic_load(&d.hval[hs], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (tb == kNone || tb >= d.cap_b) continue;
    int64_t TB[N];
    unpack_key<N>(d.key[tb], TB);
    smax = fmax(smax, add_cells<N, MODEL>(d, TB, tb, bits, lane, &ncreated));
  }
  if (lane == 0 && smax > 0.0) atomicMax(&sb->smax_bits, double_to_bits(smax));
  if (lane == 0 && ncreated > 0) atomicAdd(&sb->inserted, ncreated);
}
template <int N, int MODEL, typename Real>
__global__ __launch_bounds__(kWG) void k_grow_fix(Dev<Real> d) {
  grow_fix_body<N, MODEL, Real>(d, hw_slot());
}

// ---------------------------------------------------------------------------
// Flux passes
// ---------------------------------------------------------------------------
// Pass A computes the corrected states Q_l of every cell and stores them; pass
// B recomputes its own cells' Q_l (it holds every input already) and reads
// from neighbour bricks only the face layer of Q_l that its faces need.  Q_l
// rows are stored with the coordinate field of dimension l moved to the top
// lane bits, so that a face layer (a_l fixed) is one contiguous block of
// 64 / side values and a neighbour read touches only those cache lines.
//
// Both passes fetch the next brick's links while computing the current one,
// then load in two phases so the memory round trips overlap: every neighbour
// row first, issued unconditionally (a missing neighbour reads the permanently
// empty brick at index cap_b), then the arithmetic.

// Position of lane `lane`'s cell in a stored Q_l row.
template <int N, int L>
__device__ __forceinline__ int qpos(int lane) {
  constexpr int off = brick_off(N, L), bits = brick_bits(N, L);
  const int low = lane & ((1 << off) - 1);
  const int a = (lane >> off) & ((1 << bits) - 1);
  const int high = lane >> (off + bits);
  return low | (high << off) | (a << (6 - bits));
}
// Lane of the cell with the same coordinates as `lane` except a_J = v.
template <int N, int J>
__device__ __forceinline__ int lane_with(int lane, int v) {
  constexpr int off = brick_off(N, J), field = (brick_side(N, J) - 1) << off;
  return (lane & ~field) | (v << off);
}

// Value at distance Dd = +-1 along J when the cells of the neighbour brick
// that a boundary lane needs were loaded at that lane ("face" holds, for a
// lane with a_J at the boundary, the neighbour cell itself): boundary lanes
// take the loaded value, the others a shuffle of this brick's own values.
template <int N, int J, int Dd, typename T>
__device__ __forceinline__ T nbface(T own_shuffled, T face) {
  return lane_in(Dir<N, J, Dd>::out) ? face : own_shuffled;
}
template <int N, int J, int Dd, typename T>
__device__ __forceinline__ T own_shift(T own, int lane) {
  constexpr int side = brick_side(N, J), stride = brick_stride(N, J);
  if constexpr (side == 2)
    return xor_shfl<stride>(own);
  else
    return __shfl(own, rot_lane<N>(lane, J, Dd));
}

// Load through the constant address space: for a wave-uniform address this is
// a scalar load.  Only for data that no kernel writes while the reading kernel
// runs (brick masks during the flux passes).
template <typename T>
__device__ __forceinline__ T load_const(const T* p) {
  return *(const __attribute__((address_space(4))) T*)(p);
}

// The Dev block of a plain launch: its only argument, at the start of the
// kernel-argument segment.
template <typename Real>
__device__ __forceinline__ const Dev<Real>* kernarg_dev() {
  return (const Dev<Real>*)__builtin_amdgcn_kernarg_segment_ptr();
}

// Cell widths and grid origin read again from the grid's Dev block (the
// kernel arguments, or its copy in device memory).  Called inside a loop, it
// costs a few scalar loads (constant cache) per iteration; held across the
// loop, the values are spilled from the full scalar register file and read
// back with one vector-unit instruction per register on every use.
template <typename Real>
__device__ __forceinline__ void reload_geometry(Dev<Real>& g, const Dev<Real>* src) {
  const char* kp = reinterpret_cast<const char*>(src);
  asm volatile("" : "+s"(kp));  // not hoisted out of the loop
  const double* hp = reinterpret_cast<const double*>(kp + offsetof(Dev<Real>, h));
  const double* mp = reinterpret_cast<const double*>(kp + offsetof(Dev<Real>, mean));
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    g.h[j] = load_const(hp + j);
    g.mean[j] = load_const(mp + j);
  }
}

// A wave-uniform value computed by vector instructions, moved to scalar
// registers (keeps per-kernel constants out of the vector register file).
__device__ __forceinline__ double to_sgpr(double v) {
  const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
  const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float to_sgpr(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// Raw buffer loads from one brick row: the row's base and size form a scalar
// buffer descriptor, so per-lane addressing is a 32-bit byte offset, and an
// offset at or past the size (kOob) returns 0 without touching memory.
constexpr uint32_t kOob = 0x80000000u;
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const void* row, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(row), 0, static_cast<int>(bytes), 0x00020000);
}
__device__ __forceinline__ double row_load(__amdgpu_buffer_rsrc_t r, uint32_t off, double) {
  const u32x2_t v = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
  return __hiloint2double(static_cast<int>(v.y), static_cast<int>(v.x));
}
__device__ __forceinline__ float row_load(__amdgpu_buffer_rsrc_t r, uint32_t off, float) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

// A copy of v that the compiler cannot see through (no instruction emitted).
template <typename T>
__device__ __forceinline__ T opaque(T v) {
  asm volatile("" : "+v"(v));
  return v;
}

// acc + a * b (acc - a * b with NEG) in the lanes of the wave-uniform lane
// mask `lanes`, acc in the others.  The FMA runs with the execution mask
// narrowed to those lanes (lanes already inactive stay so), which does the
// work of a select without its vector instructions (two for a double).
template <bool NEG>
__device__ __forceinline__ double fma_lanes(u64 lanes, double a, double b, double acc) {
  u64 saved;
  if constexpr (NEG)
    asm("s_and_saveexec_b64 %1, %2\n\tv_fma_f64 %0, -%3, %4, %0\n\ts_mov_b64 exec, %1"
        : "+v"(acc), "=&s"(saved)
        : "s"(lanes), "v"(a), "v"(b)
        : "scc");
  else
    asm("s_and_saveexec_b64 %1, %2\n\tv_fma_f64 %0, %3, %4, %0\n\ts_mov_b64 exec, %1"
        : "+v"(acc), "=&s"(saved)
        : "s"(lanes), "v"(a), "v"(b)
        : "scc");
  return acc;
}
template <bool NEG>
__device__ __forceinline__ float fma_lanes(u64 lanes, float a, float b, float acc) {
  u64 saved;
  if constexpr (NEG)
    asm("s_and_saveexec_b64 %1, %2\n\tv_fma_f32 %0, -%3, %4, %0\n\ts_mov_b64 exec, %1"
        : "+v"(acc), "=&s"(saved)
        : "s"(lanes), "v"(a), "v"(b)
        : "scc");
  else
    asm("s_and_saveexec_b64 %1, %2\n\tv_fma_f32 %0, %3, %4, %0\n\ts_mov_b64 exec, %1"
        : "+v"(acc), "=&s"(saved)
        : "s"(lanes), "v"(a), "v"(b)
        : "scc");
  return acc;
}

// Transverse fluctuation T_j of one cell (see the gather form above); the
// forward term only where the +e_j neighbour is in the grid (lanes `ep`).
// Both flux passes compute it with this one function, so the corrected states
// pass A stores and pass B recomputes for its own cells are the same bits.
template <typename Real>
__device__ __forceinline__ Real t_term(Real p0, Real pm, Real pp, u64 ep, Real ub, Real uf) {
  return fma_lanes<false>(ep, rneg(uf), pp - p0, rpos(ub) * (p0 - pm));
}
// Q_l = P - sum_{j != l} c_j T_j, accumulated term by term so that Q_l is
// exactly P when every transverse T_j vanishes (with the threshold at zero,
// an exact zero decides whether a cell grows).
template <int N, typename Real>
__device__ __forceinline__ void q_from_t(Real p0, const Real* c, const Real* T, Real* q) {
#pragma unroll
  for (int l = 0; l < N; ++l) {
    Real v = p0;
#pragma unroll
    for (int j = 0; j < N; ++j)
      if (j != l) v = v - c[j] * T[j];
    q[l] = v;
  }
}

// ---------------------------------------------------------------------------
// LDS staging of pass A's inputs.  Each wave owns a slice of LDS holding, for
// the brick it computes next, its own density row and the cells that each
// axis neighbour offers across the shared face.  The slice is filled by
// load-to-LDS global loads (16 bytes per lane, no vector registers held while
// they are in flight), issued for the next brick as soon as the current
// brick's values have been read out, so the memory round trip overlaps the
// current brick's arithmetic.
//
// Slot 0 is the own row; slot 1 + 2j + s what the brick at (s ? +1 : -1) e_j
// offers: its face layer next to this brick (a_j = side - 1 below, 0 above)
// when that layer is made of whole 16-byte chunks, else its whole row.  A face
// layer is stored compacted: the cell at in-brick position x sits at x with
// the field of a_j removed.
// ---------------------------------------------------------------------------
template <int N, typename Real>
struct FaceStage {
  static constexpr int kCpc = 16 / static_cast<int>(sizeof(Real));  // cells per chunk
  static constexpr int kRowChunks = kLanes / kCpc;
  __host__ __device__ static constexpr bool layer(int j) { return brick_stride(N, j) >= kCpc; }
  __host__ __device__ static constexpr int chunks(int j) { return layer(j) ? kRowChunks / brick_side(N, j) : kRowChunks; }
  __host__ __device__ static constexpr int start(int slot) {
    int c = slot > 0 ? kRowChunks : 0;
    for (int k = 1; k < slot; ++k) c += chunks((k - 1) >> 1);
    return c;
  }
  static constexpr int kChunks = start(2 * N + 1);
  static constexpr int kInsts = (kChunks + kLanes - 1) / kLanes;
  static constexpr int kBytes = kChunks * 16;
  // Lanes of copy instruction t that copy a chunk of the brick's own row, and
  // lanes that copy nothing (past the last chunk).
  __host__ __device__ static constexpr u64 own_lanes(int t) {
    u64 m = 0;
    for (int l = 0; l < kLanes; ++l)
      if (t * kLanes + l < kRowChunks) m |= 1ull << l;
    return m;
  }
  __host__ __device__ static constexpr u64 idle_lanes(int t) {
    u64 m = 0;
    for (int l = 0; l < kLanes; ++l)
      if (t * kLanes + l >= kChunks) m |= 1ull << l;
    return m;
  }
};

// What lane `lane` copies in load-to-LDS instruction t: the link lane of the
// source brick in the meta word (-1: the brick itself, -2: nothing) and the
// byte offset of its chunk in that brick's row.
struct StageLane {
  int link;
  uint32_t off;
};
template <int N, typename Real>
__device__ __forceinline__ StageLane stage_lane(int t, int lane) {
  using F = FaceStage<N, Real>;
  const int c = t * kLanes + lane;
  StageLane r{c < F::kRowChunks ? -1 : -2, static_cast<uint32_t>(c) * 16u};
  static_for<2 * N>([&](auto Kc) {
    constexpr int k = decltype(Kc)::value, j = k >> 1, s = k & 1;
    constexpr int lo = F::start(1 + k), hi = F::start(2 + k);
    if (c >= lo && c < hi) {
      const int q = c - lo;
      r.link = k;
      if constexpr (F::layer(j)) {
        constexpr int off = brick_off(N, j), bits = brick_bits(N, j), v = s ? 0 : brick_side(N, j) - 1;
        const int y = q * F::kCpc;
        const int x = (y & ((1 << off) - 1)) | (v << off) | ((y >> off) << (off + bits));
        r.off = static_cast<uint32_t>(x) * sizeof(Real);
      } else {
        r.off = static_cast<uint32_t>(q) * 16u;
      }
    }
  });
  return r;
}

typedef __attribute__((address_space(3))) char lds_char;
// An LDS address the compiler cannot see through: values derived from it
// (the per-copy LDS targets) are formed where they are used instead of being
// hoisted out of the brick loop into scalar registers that then spill.
__device__ __forceinline__ lds_char* lds_opaque(char* p) {
  uint32_t a = static_cast<uint32_t>(reinterpret_cast<uintptr_t>((lds_char*)p));
  asm volatile("" : "+s"(a));
  return (lds_char*)static_cast<uintptr_t>(a);
}
// Starts the copies of brick b's staged inputs (mv: b's meta word) into the
// wave's slice.  Missing neighbours read the permanently empty brick cap_b.
template <int N, typename Real>
__device__ __forceinline__ void stage_issue(const Real* P, uint32_t b, uint32_t mv, uint32_t cap_b, const StageLane* pl,
                                            char* slice_in) {
  using F = FaceStage<N, Real>;
  lds_char* slice = lds_opaque(slice_in);
  static_for<F::kInsts>([&](auto Tc) {
    constexpr int t = decltype(Tc)::value;
    constexpr u64 own = F::own_lanes(t), idle = F::idle_lanes(t);
    uint32_t idx = b;
    if constexpr (own != ~0ull) {
      idx = static_cast<uint32_t>(__shfl(static_cast<int>(mv), pl[t].link > 0 ? pl[t].link : 0));
      if constexpr (own != 0ull) idx = lane_in(own) ? b : idx;
      idx = idx == kNone ? cap_b : idx;
    }
    const char* src = reinterpret_cast<const char*>(P + static_cast<size_t>(idx) * kLanes) + pl[t].off;
    if (idle == 0ull || lane_in(~idle))
      __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)(slice + t * kLanes * 16), 16, 0, 0);
  });
}

// Byte position in the slice of the cell that the brick at (S ? +1 : -1) e_J
// offers to lane `lane`.
template <int N, typename Real, int J, int S>
__device__ __forceinline__ uint32_t stage_pos(int lane) {
  using F = FaceStage<N, Real>;
  constexpr int off = brick_off(N, J), bits = brick_bits(N, J);
  constexpr uint32_t base = static_cast<uint32_t>(F::start(1 + 2 * J + S)) * 16u;
  if constexpr (F::layer(J)) {
    const int y = (lane & ((1 << off) - 1)) | ((lane >> (off + bits)) << off);
    return base + static_cast<uint32_t>(y) * sizeof(Real);
  } else {
    return base + static_cast<uint32_t>(lane_with<N, J>(lane, S ? 0 : brick_side(N, J) - 1)) * sizeof(Real);
  }
}
template <typename Real>
__device__ __forceinline__ Real slice_read(const char* slice, uint32_t pos) {
  return *reinterpret_cast<const Real*>(slice + pos);
}
// The compiler does not order LDS reads against load-to-LDS copies, so the
// two waits are explicit and are also compiler barriers for memory accesses:
// copies into the slice have landed before it is read, and its reads have
// returned before it is refilled.
__device__ __forceinline__ void wait_stage_landed() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }
__device__ __forceinline__ void wait_lds_reads() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// Flux pass A: transverse fluctuations and corrected states Q_l.
template <int N, int MODEL, typename Real>
__device__ __forceinline__ void flux_a_body(const Dev<Real>& d, const Dev<Real>* dsrc, Slot sl) {
  const Scalars* sb = d.sb;
  // The scalar block is written only between passes: read it as constant.
  if (!load_const(&sb->run)) return;
  const uint32_t nb = min(load_const(&sb->nb), d.cap_b);
  const Real* P = load_const(&sb->cur) ? d.P1 : d.P0;
  const double dt = load_const(&sb->dt);
  Real c[N];
#pragma unroll
  for (int j = 0; j < N; ++j) c[j] = static_cast<Real>(dt / (2.0 * d.h[j]));
  const int lane = lane_id();
  using F = FaceStage<N, Real>;
  __shared__ __align__(16) char stage_all[kWavesPerWG][F::kBytes];
  char* slice = stage_all[__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)];
  StageLane pl[F::kInsts];
#pragma unroll
  for (int t = 0; t < F::kInsts; ++t) pl[t] = stage_lane<N, Real>(t, lane);
  const WaveRange rg = wave_range(nb, sl);
  // The slice holds brick b's inputs while b is computed; meta holds b's
  // links and meta_n those of the next brick.
  const MetaLane ml = meta_lane<N>(d, lane);
  uint32_t meta = meta_fetch<N>(ml, rg.begin < rg.end ? rg.begin : kNone);
  if (rg.begin < rg.end) stage_issue<N>(P, rg.begin, meta, d.cap_b, pl, slice);
  uint32_t meta_n = meta_fetch<N>(ml, rg.begin + rg.step < rg.end ? rg.begin + rg.step : kNone);
  // A brick's Q_l face layers are stored one iteration late, after the next
  // copies have been issued: the wait for those copies then finds the stores
  // long done instead of waiting for their completion.
  Real qs[N];
  // Wave-uniform: bit 2l set when brick bprev stores its Q_l layer next to
  // the +e_l face, bit 2l + 1 when it stores the one next to the -e_l face.
  uint32_t kb = 0;
  uint32_t bprev = kNone;
  auto store_q = [&](uint32_t bq) {
    Real* Qb = d.Q + static_cast<size_t>(bq) * N * kLanes;
    static_for<N>([&](auto Lc) {
      constexpr int l = decltype(Lc)::value;
      const u64 lanes = ((kb >> (2 * l)) & 1u ? Dir<N, l, 1>::out : 0ull) | ((kb >> (2 * l)) & 2u ? Dir<N, l, -1>::out : 0ull);
      if (lane_in(lanes)) Qb[l * kLanes + qpos<N, l>(lane)] = qs[l];
    });
  };
  for (uint32_t b = rg.begin; b < rg.end; b += rg.step) {
    const BrickMeta<N> bm = meta_unpack<N>(meta);
    wait_stage_landed();
    const Real p0 = slice_read<Real>(slice, static_cast<uint32_t>(lane) * sizeof(Real));
    Real Fm[N], Fp[N];
    static_for<N>([&](auto Jc) {
      constexpr int j = decltype(Jc)::value;
      Fm[j] = slice_read<Real>(slice, stage_pos<N, Real, j, 0>(lane));
      Fp[j] = slice_read<Real>(slice, stage_pos<N, Real, j, 1>(lane));
    });
    wait_lds_reads();
    const uint32_t bn = b + rg.step;
    if (bn < rg.end) stage_issue<N>(P, bn, meta_n, d.cap_b, pl, slice);
    meta = meta_n;
    meta_n = meta_fetch<N>(ml, bn + rg.step < rg.end ? bn + rg.step : kNone);
    if (bprev != kNone) store_q(bprev);
    // The masks after this step's grow are the next step's start masks.
    if (lane == 0) d.abv[b] = bm.mask;
    Dev<Real> dv = d;
    reload_geometry(dv, dsrc);
    u64 mm[N], mp[N];
    static_for<N>([&](auto Jc) {
      constexpr int j = decltype(Jc)::value;
      mm[j] = load_const(d.mask + (bm.bm[j] != kNone ? bm.bm[j] : d.cap_b));
      mp[j] = load_const(d.mask + (bm.bp[j] != kNone ? bm.bp[j] : d.cap_b));
    });
    int64_t B[N];
    unpack_key<N>(bm.key, B);
    int32_t ii[N];
    double xc[N];
    cell_of<N>(dv, B, lane, ii, xc);
    Real T[N];
    uint32_t kn = 0;  // the next value of kb
    static_for<N>([&](auto Jc) {
      constexpr int j = decltype(Jc)::value;
      Real pm, pp;
      if constexpr (brick_side(N, j) == 2) {
        const Real sh = own_shift<N, j, 1>(p0, lane);
        pm = nbface<N, j, -1>(sh, Fm[j]);
        pp = nbface<N, j, 1>(sh, Fp[j]);
      } else {
        pm = nbface<N, j, -1>(own_shift<N, j, -1>(p0, lane), Fm[j]);
        pp = nbface<N, j, 1>(own_shift<N, j, 1>(p0, lane), Fp[j]);
      }
      const u64 ep = present_lanes<N, j, 1>(bm.mask, mp[j]);
      const Real ub = static_cast<Real>(face_vel<MODEL, N>(dv, xc, ii, j));
      const Real uf = static_cast<Real>(face_vel_fwd<MODEL, N>(dv, xc, ii, j));
      T[j] = t_term(p0, pm, pp, ep, ub, uf);
      // A face layer's Q_l is read across the brick face only by the
      // downwind neighbour: the +e_j brick when the forward face velocity is
      // positive, the -e_j brick when the backward one is negative, and only
      // where the cell across the face is in the grid (a face with a missing
      // side carries no flux).  Stored per whole face layer (full cache
      // lines, no partial writes).
      const u64 across = (present_lanes<N, j, 1>(bm.mask, mp[j]) & Dir<N, j, 1>::out) |
                         (present_lanes<N, j, -1>(bm.mask, mm[j]) & Dir<N, j, -1>::out);
      const u64 want = ballot((lane_in(Dir<N, j, 1>::out) && uf > Real(0)) || (lane_in(Dir<N, j, -1>::out) && ub < Real(0))) & bm.mask & across;
      kn |= ((want & Dir<N, j, 1>::out) ? 1u : 0u) << (2 * j);
      kn |= ((want & Dir<N, j, -1>::out) ? 2u : 0u) << (2 * j);
    });
    // Lanes of absent cells in a stored layer store their Q_l too: pass B
    // uses a face value only where the cells on both sides are in the grid.
    q_from_t<N>(p0, c, T, qs);
    kb = kn;
    bprev = b;
  }
  if (bprev != kNone) store_q(bprev);
}
template <int N, int MODEL, typename Real>
__global__ __launch_bounds__(kWG, kFluxWavesPerEU) void k_flux_a(Dev<Real> d) {
  flux_a_body<N, MODEL, Real>(d, kernarg_dev<Real>(), hw_slot());
}

// Flux pass B: face fluxes, high-resolution term, conservative update.
template <int N, int MODEL, typename Real>
__device__ __forceinline__ void flux_b_body(const Dev<Real>& d, const Dev<Real>* dsrc, Slot sl) {
  const Scalars* sb = d.sb;
  // The scalar block is written only between passes: read it as constant.
  if (!load_const(&sb->run)) return;
  const uint32_t nb = min(load_const(&sb->nb), d.cap_b);
  const uint32_t cur = load_const(&sb->cur);
  const Real* P = cur ? d.P1 : d.P0;
  Real* Pn = cur ? d.P0 : d.P1;
  const double dt = load_const(&sb->dt);
  Real dth[N], c[N];
#pragma unroll
  for (int j = 0; j < N; ++j) {
    dth[j] = static_cast<Real>(dt / d.h[j]);
    c[j] = static_cast<Real>(dt / (2.0 * d.h[j]));
  }
  const bool hr = d.limiter != 0;
  const int lane = lane_id();
  double vmax = 0.0, vsum = 0.0;
  uint32_t ncells = 0;  // wave-uniform
  const WaveRange rg = wave_range(nb, sl);
  const MetaLane ml = meta_lane<N>(d, lane);
  uint32_t meta = meta_fetch<N>(ml, rg.begin < rg.end ? rg.begin : kNone);
  for (uint32_t b = rg.begin; b < rg.end; b += rg.step) {
    const BrickMeta<N> bm = meta_unpack<N>(meta);
    const size_t o = static_cast<size_t>(b) * kLanes + lane;
    const Real p0 = P[o];
    Dev<Real> dg = d;
    reload_geometry(dg, dsrc);
    int64_t B[N];
    unpack_key<N>(bm.key, B);
    int32_t ii[N];
    double xc[N];
    cell_of<N>(dg, B, lane, ii, xc);
    Real ub[N], uf[N];
    static_for<N>([&](auto Lc) {
      constexpr int l = decltype(Lc)::value;
      ub[l] = static_cast<Real>(face_vel<MODEL, N>(dg, xc, ii, l));
      uf[l] = static_cast<Real>(face_vel_fwd<MODEL, N>(dg, xc, ii, l));
    });
    Real Pm[N], Pp[N], Qm[N], Qp[N];
    u64 mm[N], mp[N];
    // Full neighbour density rows (the high-resolution term reads distance 2).
    // Q_l only in the face layer and only where the face velocity points out
    // of the neighbour; other lanes load nothing (out-of-range offset).
    static_for<N>([&](auto Lc) {
      constexpr int l = decltype(Lc)::value;
      constexpr int side = brick_side(N, l);
      constexpr uint32_t kRow = kLanes * sizeof(Real);
      const uint32_t im = bm.bm[l] != kNone ? bm.bm[l] : d.cap_b, ip = bm.bp[l] != kNone ? bm.bp[l] : d.cap_b;
      const bool need_m = lane_in(Dir<N, l, -1>::out) && ub[l] > Real(0);
      const bool need_p = lane_in(Dir<N, l, 1>::out) && uf[l] < Real(0);
      Pm[l] = row_load(row_rsrc(P + static_cast<size_t>(im) * kLanes, kRow), lane * sizeof(Real), Real(0));
      Pp[l] = row_load(row_rsrc(P + static_cast<size_t>(ip) * kLanes, kRow), lane * sizeof(Real), Real(0));
      Qm[l] = row_load(row_rsrc(d.Q + (static_cast<size_t>(im) * N + l) * kLanes, kRow),
                       need_m ? qpos<N, l>(lane_with<N, l>(lane, side - 1)) * sizeof(Real) : kOob, Real(0));
      Qp[l] = row_load(row_rsrc(d.Q + (static_cast<size_t>(ip) * N + l) * kLanes, kRow),
                       need_p ? qpos<N, l>(lane_with<N, l>(lane, 0)) * sizeof(Real) : kOob, Real(0));
      mm[l] = load_const(d.mask + im);
      mp[l] = load_const(d.mask + ip);
    });
    const uint32_t bn = b + rg.step;
    meta = meta_fetch<N>(ml, bn < rg.end ? bn : kNone);
    // This brick's own corrected states, as pass A computed them.
    Real T[N];
    static_for<N>([&](auto Lc) {
      constexpr int l = decltype(Lc)::value;
      T[l] = t_term(p0, nbval<N, l, -1>(p0, Pm[l], lane), nbval<N, l, 1>(p0, Pp[l], lane),
                    present_lanes<N, l, 1>(bm.mask, mp[l]), ub[l], uf[l]);
    });
    Real q[N];
    q_from_t<N>(p0, c, T, q);
    // The distance-1 neighbour values are shuffled again below rather than
    // kept live across both loops (register pressure); the opaque copy of P
    // stops the compiler from merging the two computations.
    const Real p0r = opaque(p0);
    Real acc = p0;
    static_for<N>([&](auto Lc) {
      constexpr int l = decltype(Lc)::value;
      // Faces of cells in the grid whose other side is in the grid too; the
      // others carry no flux, and absent cells keep their 0.
      const u64 em = present_lanes<N, l, -1>(bm.mask, mm[l]) & bm.mask;
      const u64 ep = present_lanes<N, l, 1>(bm.mask, mp[l]) & bm.mask;
      const Real pm1 = nbval<N, l, -1>(p0r, Pm[l], lane);
      const Real pp1 = nbval<N, l, 1>(p0r, Pp[l], lane);
      Real qm, qp;
      if constexpr (brick_side(N, l) == 2) {
        const Real sh = own_shift<N, l, 1>(q[l], lane);
        qm = nbface<N, l, -1>(sh, Qm[l]);
        qp = nbface<N, l, 1>(sh, Qp[l]);
      } else {
        qm = nbface<N, l, -1>(own_shift<N, l, -1>(q[l], lane), Qm[l]);
        qp = nbface<N, l, 1>(own_shift<N, l, 1>(q[l], lane), Qp[l]);
      }
      // Upwind states: a neighbour's stored Q_l is read only where the face
      // velocity strictly points out of it (pass A stores no other face
      // values, and a zero velocity must not meet an unwritten one).
      Real fb = ub[l] * (ub[l] > Real(0) ? qm : q[l]);
      Real ff = uf[l] * (uf[l] < Real(0) ? qp : q[l]);
      if (hr) {
        const Real pm2 = nbval<N, l, -2>(p0r, Pm[l], lane);
        const Real pp2 = nbval<N, l, 2>(p0r, Pp[l], lane);
        fb += hr_term(ub[l], dth[l], p0r - pm1, ub[l] > Real(0) ? pm1 - pm2 : pp1 - p0r);
        ff += hr_term(uf[l], dth[l], pp1 - p0r, uf[l] > Real(0) ? p0r - pm1 : pp2 - pp1);
      }
      acc = fma_lanes<false>(em, dth[l], fb, acc);
      acc = fma_lanes<true>(ep, dth[l], ff, acc);
    });
    // An absent cell's acc is its stored P, which is 0.
    const Real out = acc;
    Pn[o] = out;
    // Absent cells hold 0: they leave the sum unchanged and cannot raise the
    // maximum above its start value 0.
    vmax = fmax(vmax, static_cast<double>(out));
    vsum += static_cast<double>(out);
    ncells += static_cast<uint32_t>(__builtin_popcountll(bm.mask));
  }
  wg_store3(vmax, vsum, lane == 0 ? static_cast<double>(ncells) : 0.0, d.dpart, sl.wg);
}
template <int N, int MODEL, typename Real>
__global__ __launch_bounds__(kWG, sizeof(Real) == 8 ? kFluxBWavesPerEU64 : kFluxBWavesPerEU32) void k_flux_b(Dev<Real> d) {
  flux_b_body<N, MODEL, Real>(d, kernarg_dev<Real>(), hw_slot());
}

// ---------------------------------------------------------------------------
// One time step of several grids per launch (MultiGrids): workgroup w serves
// the grid whose run [wg0[r], wg0[r + 1]) holds it, with that grid's own
// workgroup index and count, so every grid computes exactly what its plain
// launches compute.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t multi_grid(const MultiGrids& m, uint32_t w) {
  uint32_t r = 0;
  while (r + 1 < m.R && m.wg0[r + 1] <= w) ++r;
  return r;
}
// Grid r's Dev block, read through the constant address space: the copy in
// device memory never changes while kernels run, and saying so lets its fields
// live in scalar registers like kernel arguments.
template <typename Real>
__device__ __forceinline__ Dev<Real> multi_dev(const MultiGrids& m, uint32_t r) {
  static_assert(sizeof(Dev<Real>) % 8 == 0, "Dev is copied in 8-byte words");
  constexpr int kWords = sizeof(Dev<Real>) / 8;
  const u64* src = static_cast<const u64*>(m.dev[r]);
  u64 w[kWords];
#pragma unroll
  for (int k = 0; k < kWords; ++k) w[k] = load_const(src + k);  // unused words are never loaded
  Dev<Real> d;
  __builtin_memcpy(&d, w, sizeof(d));
  return d;
}
__device__ __forceinline__ Slot multi_slot(const MultiGrids& m, uint32_t r) {
  return Slot{blockIdx.x - m.wg0[r], m.wg0[r + 1] - m.wg0[r]};
}

// One workgroup per grid.
template <typename Real>
__global__ void k_scalar_multi(MultiGrids m, int op) {
  scalar_op(multi_dev<Real>(m, blockIdx.x), op, 0.0);
}
template <typename Real>
__global__ void k_final_step_multi(MultiGrids m) {
  final_step(multi_dev<Real>(m, blockIdx.x), m.wg0[blockIdx.x + 1] - m.wg0[blockIdx.x]);
}
// wg0[R] workgroups.
template <int N, int MODEL, typename Real>
__global__ __launch_bounds__(kWG, 4) void k_grow_multi(MultiGrids m) {
  const uint32_t r = multi_grid(m, blockIdx.x);
  grow_body<N, MODEL, Real>(multi_dev<Real>(m, r), multi_slot(m, r));
}
template <int N, int MODEL, typename Real>
__global__ __launch_bounds__(kWG) void k_grow_fix_multi(MultiGrids m) {
  const uint32_t r = multi_grid(m, blockIdx.x);
  grow_fix_body<N, MODEL, Real>(multi_dev<Real>(m, r), multi_slot(m, r));
}
template <int N, int MODEL, typename Real>
__global__ __launch_bounds__(kWG, kFluxWavesPerEU) void k_flux_a_multi(MultiGrids m) {
  const uint32_t r = multi_grid(m, blockIdx.x);
  flux_a_body<N, MODEL, Real>(multi_dev<Real>(m, r), static_cast<const Dev<Real>*>(m.dev[r]), multi_slot(m, r));
}
template <int N, int MODEL, typename Real>
__global__ __launch_bounds__(kWG, sizeof(Real) == 8 ? kFluxBWavesPerEU64 : kFluxBWavesPerEU32) void k_flux_b_multi(
    MultiGrids m) {
  const uint32_t r = multi_grid(m, blockIdx.x);
  flux_b_body<N, MODEL, Real>(multi_dev<Real>(m, r), static_cast<const Dev<Real>*>(m.dev[r]), multi_slot(m, r));
}

// ---------------------------------------------------------------------------
// Prune (Sec. 3.3 upwind rule, Algorithm 3)
// ---------------------------------------------------------------------------
template <int N, typename Real>
__global__ __launch_bounds__(kWG) void k_prune_above(Dev<Real> d) {
  if (!d.sb->prun) return;
  const Real* P = cur_p(d);
  const Real pstar = static_cast<Real>(d.thresh_rel * d.sb->maxp);
  const int lane = lane_id();
  const WaveRange rg = wave_range(nb_of(d));
  for (uint32_t b = rg.begin; b < rg.end; b += rg.step) {
    const u64 m = d.mask[b];
    const bool a = ((m >> lane) & 1ull) && (P[static_cast<size_t>(b) * kLanes + lane] >= pstar);
    const u64 A = ballot(a);
    if (lane == 0) d.abv[b] = A;
  }
}

template <int N, int MODEL, typename Real>
__global__ __launch_bounds__(kWG) void k_prune_mark(Dev<Real> d) {
  Scalars* sb = d.sb;
  if (!sb->prun) return;
  const int lane = lane_id();
  double smax = 0.0;
  const WaveRange rg = wave_range(nb_of(d));
  for (uint32_t b = rg.begin; b < rg.end; b += rg.step) {
    const u64 m = d.mask[b];
    const u64 A = d.abv[b];
    const uint32_t axl = axis_links<N>(d, b, lane);
    const u64 below = m & ~A;  // present cells with P < p*
    u64 keep = A;
    int64_t B[N];
    unpack_key<N>(d.key[b], B);
    int32_t ii[N];
    double xc[N];
    cell_of<N>(d, B, lane, ii, xc);
    if (below != 0ull) {
      // Above-threshold lanes of every target brick, one target per lane.
      uint32_t t0 = resolve_target<N>(d, b, lane, axl, true);
      uint32_t t1 = resolve_target<N>(d, b, lane + 64, axl, true);
      if (t0 == kNone && lane < n_targets(N)) {
        int j = 0, s = 0, l = 0, r = 0;
        if (target_kind<N>(lane, &j, &s, &l, &r) == 2) {
          int64_t TB[N];
#pragma unroll
          for (int q = 0; q < N; ++q) TB[q] = B[q] + (q == j ? s : 0) + (q == l ? r : 0);
          if (brick_in_range<N>(TB)) t0 = hash_find(d, pack_key<N>(TB));
        }
      }
      if (t1 == kNone && lane + 64 < n_targets(N)) {
        int j = 0, s = 0, l = 0, r = 0;
        if (target_kind<N>(lane + 64, &j, &s, &l, &r) == 2) {
          int64_t TB[N];
#pragma unroll
          for (int q = 0; q < N; ++q) TB[q] = B[q] + (q == j ? s : 0) + (q == l ? r : 0);
          if (brick_in_range<N>(TB)) t1 = hash_find(d, pack_key<N>(TB));
        }
      }
      const u64 a0 = (t0 != kNone && t0 < d.cap_b) ? d.abv[t0] : 0ull;
      const u64 a1 = (t1 != kNone && t1 < d.cap_b) ? d.abv[t1] : 0ull;
      const bool bl = (below >> lane) & 1ull;
      u64 U[N], D[N];  // below lanes with an upwind neighbour at +e_j / -e_j
#pragma unroll
      for (int j = 0; j < N; ++j) {
        U[j] = ballot(bl && face_vel_fwd<MODEL, N>(d, xc, ii, j) < 0.0);
        D[j] = ballot(bl && face_vel<MODEL, N>(d, xc, ii, j) > 0.0);
      }
      u64 k2 = 0ull;
      static_for<N>([&](auto Jc) {
        constexpr int j = decltype(Jc)::value;
        static_for<2>([&](auto Sc) {
          constexpr int si = decltype(Sc)::value;
          using Dj = Dir<N, j, si ? 1 : -1>;
          const u64 src = si ? U[j] : D[j];
          if (src == 0ull) return;
          k2 |= src & Dj::in & lshc<-Dj::sh_in>(A);
          k2 |= src & Dj::out & lshc<-Dj::sh_out>(target_word(a0, a1, 1 + 2 * j + si));
        });
      });
      static_for<N*(N - 1) / 2>([&](auto Pc) {
        constexpr int pair = decltype(Pc)::value;
        constexpr int j = pair_j(N, pair), l = pair_l(N, pair);
        static_for<4>([&](auto Cc) {
          constexpr int si = decltype(Cc)::value >> 1, ri = decltype(Cc)::value & 1;
          using Dj = Dir<N, j, si ? 1 : -1>;
          using Dl = Dir<N, l, ri ? 1 : -1>;
          const u64 src = (si ? U[j] : D[j]) & (ri ? U[l] : D[l]);
          if (src == 0ull) return;
          k2 |= src & Dj::in & Dl::in & lshc<-(Dj::sh_in + Dl::sh_in)>(A);
          k2 |= src & Dj::out & Dl::in & lshc<-(Dj::sh_out + Dl::sh_in)>(target_word(a0, a1, 1 + 2 * j + si));
          k2 |= src & Dj::in & Dl::out & lshc<-(Dj::sh_in + Dl::sh_out)>(target_word(a0, a1, 1 + 2 * l + ri));
          k2 |= src & Dj::out & Dl::out &
                lshc<-(Dj::sh_out + Dl::sh_out)>(target_word(a0, a1, 1 + 2 * N + 4 * pair + 2 * si + ri));
        });
      });
      keep |= k2 & below;
    }
    if (lane == 0) d.mask[b] = keep;
    if ((keep >> lane) & 1ull) smax = fmax(smax, cell_speed<MODEL, N>(d, xc, ii));
  }
  smax = wave_max(smax);
  if (lane == 0 && smax > 0.0) atomicMax(&sb->smax_bits, double_to_bits(smax));
}

// ---------------------------------------------------------------------------
// Orthant grow and prune (grow_mode 2; Sec. 3.3, Figs. 2-3): a source cell
// grows every combination of its downwind steps, at most one step per
// dimension (up to 2^n - 1 cells, more where a cell has both a +e_j and a
// -e_j downwind side), and a below-threshold cell survives a prune when any
// combination of its upwind steps reaches a cell at or above p*.  The
// candidate cells of a brick fall into the 3^n bricks at offsets in
// {-1, 0, 1}^n; the grow pass gathers them per target brick in LDS, one
// 64-bit lane mask per target, from a per-lane walk over the lane's own step
// combinations, then resolves the targets lane-parallel like the pairwise
// pass (links for axis and edge targets, the hashtable beyond).
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int pow3(int n) { return n == 0 ? 1 : 3 * pow3(n - 1); }

// Next step combination after st (digits in {-1, 0, +1}): per dimension 0,
// then +1 if allowed, then -1 if allowed, carrying into the next dimension.
// False once every combination was visited.
template <int N>
__device__ __forceinline__ bool next_steps(int* st, const bool* plus, const bool* minus) {
#pragma unroll
  for (int j = 0; j < N; ++j) {
    if (st[j] == 0 && plus[j]) {
      st[j] = 1;
      return true;
    }
    if (st[j] != -1 && minus[j]) {
      st[j] = -1;
      return true;
    }
    st[j] = 0;
  }
  return false;
}

// Where lane `lane` lands after the steps st: the target brick's offset as a
// base-3 index (digit j = offset_j + 1) and the lane in that brick.
template <int N>
__device__ __forceinline__ void step_target(int lane, const int* st, int* tidx, int* tlane) {
  int t = 0, l = 0, w = 1;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const int side = brick_side(N, j);
    const int a = ((lane >> brick_off(N, j)) & (side - 1)) + st[j];
    const int o = a < 0 ? -1 : (a >= side ? 1 : 0);
    t += (o + 1) * w;
    w *= 3;
    l |= (a - o * side) << brick_off(N, j);
  }
  *tidx = t;
  *tlane = l;
}

// Brick at base-3 offset index k from brick b (coordinates B): through the
// axis links for up to two non-zero offsets, else through the hashtable.
// kNone if it does not exist (or is not yet linked).
template <int N, typename Real>
__device__ __forceinline__ uint32_t orthant_brick(const Dev<Real>& d, uint32_t b, const int64_t* B, int k) {
  int off[N];
  int nz = 0, j0 = -1, j1 = -1;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    off[j] = k % 3 - 1;
    k /= 3;
    if (off[j] != 0) {
      j1 = j0 < 0 ? -1 : j;
      j0 = j0 < 0 ? j : j0;
      ++nz;
    }
  }
  if (nz == 0) return b;
  if (nz == 1) return nbr_of(d, b, j0, off[j0]);
  if (nz == 2) {
    uint32_t t = nbr_of(d, nbr_of(d, b, j0, off[j0]), j1, off[j1]);
    if (t == kNone) t = nbr_of(d, nbr_of(d, b, j1, off[j1]), j0, off[j0]);
    if (t != kNone) return t;
  }
  int64_t TB[N];
#pragma unroll
  for (int j = 0; j < N; ++j) TB[j] = B[j] + off[j];
  if (!brick_in_range<N>(TB)) return kNone;
  return hash_find(d, pack_key<N>(TB));
}

template <int N, int MODEL, typename Real>
__device__ __forceinline__ void grow_orthant_body(const Dev<Real>& d, Slot sl) {
  Scalars* sb = d.sb;
  if (!sb->run) return;
  const uint32_t nb_old = sb->nb_old;
  const Real* P = cur_p(d);
  const bool thr0 = !(d.thresh_rel > 0.0);
  const Real pstar = uniform(static_cast<Real>(d.thresh_rel * sb->maxp));
  const int lane = lane_id();
  constexpr int NT = pow3(N), CENTRE = (pow3(N) - 1) / 2;
  __shared__ u64 tbl_all[kWavesPerWG][NT];
  u64* tbl = tbl_all[threadIdx.x >> 6];
  double smax = 0.0;
  u64 nscan = 0, ncreated = 0;
  const WaveRange rg = wave_range(nb_old, sl);
  for (uint32_t b = rg.begin; b < rg.end; b += rg.step) {
    const u64 m = d.mask[b], dn = d.done[b];
    if ((m & ~dn) == 0ull) continue;
    const Real pv = P[static_cast<size_t>(b) * kLanes + lane];
    const bool src = ((m >> lane) & 1ull) && (thr0 ? (pv != Real(0)) : (pv >= pstar));
    const u64 S = ballot(src);
    const u64 todo = S & ~dn;
    if (todo == 0ull) continue;
    if (lane == 0) {
      d.done[b] = dn | S;
      ++nscan;
    }
    for (int k = lane; k < NT; k += kLanes) tbl[k] = 0ull;
    wave_lds_sync();
    int64_t B[N];
    unpack_key<N>(d.key[b], B);
    int32_t ii[N];
    double xc[N];
    cell_of<N>(d, B, lane, ii, xc);
    if ((todo >> lane) & 1ull) {
      bool plus[N], minus[N];
#pragma unroll
      for (int j = 0; j < N; ++j) {
        plus[j] = face_vel_fwd<MODEL, N>(d, xc, ii, j) > 0.0;
        minus[j] = face_vel<MODEL, N>(d, xc, ii, j) < 0.0;
      }
      int st[N];
#pragma unroll
      for (int j = 0; j < N; ++j) st[j] = 0;
      while (next_steps<N>(st, plus, minus)) {
        int ti, tl;
        step_target<N>(lane, st, &ti, &tl);
        __hip_atomic_fetch_or(&tbl[ti], 1ull << tl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
      }
    }
    wave_lds_sync();
    if (lane == 0) tbl[CENTRE] &= ~m;
    wave_lds_sync();
    for (int k0 = 0; k0 < NT; k0 += kLanes) {
      const int k = k0 + lane;
      const u64 bits = k < NT ? tbl[k] : 0ull;
      const uint32_t t = bits != 0ull ? orthant_brick<N>(d, b, B, k) : kNone;
      const u64 made = (bits != 0ull && t != kNone) ? bits & ~atomicOr(&d.mask[t], bits) : 0ull;
      u64 made_t = ballot(made != 0ull);
      u64 hash_t = ballot(bits != 0ull && t == kNone);
      auto target_brick = [&](int kk, int64_t* TB) {
#pragma unroll
        for (int j = 0; j < N; ++j) {
          TB[j] = B[j] + (kk % 3 - 1);
          kk /= 3;
        }
      };
      while (made_t != 0ull) {
        const int kl = __builtin_ctzll(made_t);
        made_t &= made_t - 1ull;
        const u64 mk = readlane64(made, kl);
        int64_t TB[N];
        target_brick(k0 + kl, TB);
        ncreated += static_cast<u64>(__popcll(mk));
        smax = fmax(smax, created_speed<N, MODEL>(d, TB, mk, lane));
      }
      while (hash_t != 0ull) {
        const int kl = __builtin_ctzll(hash_t);
        hash_t &= hash_t - 1ull;
        const u64 bk = readlane64(bits, kl);
        int64_t TB[N];
        target_brick(k0 + kl, TB);
        smax = fmax(smax, add_cells<N, MODEL>(d, TB, kNone, bk, lane, &ncreated));
      }
    }
    wave_lds_sync();
  }
  smax = wave_max(smax);
  if (lane == 0 && smax > 0.0) atomicMax(&sb->smax_bits, double_to_bits(smax));
  if (lane == 0 && nscan > 0) atomicAdd(&sb->grow_bricks, nscan);
  if (lane == 0 && ncreated > 0) atomicAdd(&sb->inserted, ncreated);
}
template <int N, int MODEL, typename Real>
__global__ __launch_bounds__(kWG) void k_grow_orthant(Dev<Real> d) {
  grow_orthant_body<N, MODEL, Real>(d, hw_slot());
}

// Orthant prune marks: a present cell below p* keeps its bit if any
// combination of its upwind steps (+e_j where the forward-face velocity is
// negative, -e_j where the backward-face velocity is positive) reaches a cell
// whose above-threshold bit is set.
template <int N, int MODEL, typename Real>
__global__ __launch_bounds__(kWG) void k_prune_mark_orthant(Dev<Real> d) {
  Scalars* sb = d.sb;
  if (!sb->prun) return;
  const int lane = lane_id();
  double smax = 0.0;
  const WaveRange rg = wave_range(nb_of(d));
  for (uint32_t b = rg.begin; b < rg.end; b += rg.step) {
    const u64 m = d.mask[b];
    const u64 A = d.abv[b];
    const u64 below = m & ~A;
    int64_t B[N];
    unpack_key<N>(d.key[b], B);
    int32_t ii[N];
    double xc[N];
    cell_of<N>(d, B, lane, ii, xc);
    bool kept = false;
    if ((below >> lane) & 1ull) {
      bool plus[N], minus[N];
#pragma unroll
      for (int j = 0; j < N; ++j) {
        plus[j] = face_vel_fwd<MODEL, N>(d, xc, ii, j) < 0.0;
        minus[j] = face_vel<MODEL, N>(d, xc, ii, j) > 0.0;
      }
      int st[N];
#pragma unroll
      for (int j = 0; j < N; ++j) st[j] = 0;
      while (!kept && next_steps<N>(st, plus, minus)) {
        int ti, tl;
        step_target<N>(lane, st, &ti, &tl);
        const uint32_t t = orthant_brick<N>(d, b, B, ti);
        if (t != kNone && t < d.cap_b) kept = (d.abv[t] >> tl) & 1ull;
      }
    }
    const u64 keep = A | (ballot(kept) & below);
    if (lane == 0) d.mask[b] = keep;
    if ((keep >> lane) & 1ull) smax = fmax(smax, cell_speed<MODEL, N>(d, xc, ii));
  }
  smax = wave_max(smax);
  if (lane == 0 && smax > 0.0) atomicMax(&sb->smax_bits, double_to_bits(smax));
}

// ---------------------------------------------------------------------------
// Reordering at prune: the bricks that kept a cell are sorted by the Morton
// code of their brick coordinates (removed bricks sort last), so that the
// axis neighbours of a brick sit close to it in memory and in time.  Stable
// LSD radix sort, 8-bit digits, one digit histogram per workgroup chunk.
// Scratch (in the Q region): keys A/B, values A/B, then key2/mask2 copies.
// ---------------------------------------------------------------------------
constexpr int kSortWG = 256;  // workgroups of the radix passes (chunked)

struct SortScratch {
  u64 *ka, *kb;
  uint32_t *va, *vb;
  u64 *key2, *mask2;
  uint32_t* hist;  // [256][kSortWG]
};
template <typename Real>
__device__ __forceinline__ SortScratch sort_scratch(const Dev<Real>& d) {
  const size_t cap = d.cap_b;
  u64* base = reinterpret_cast<u64*>(d.Q);
  SortScratch sc;
  sc.ka = base;
  sc.kb = base + cap;
  sc.key2 = base + 2 * cap;
  sc.mask2 = base + 3 * cap;
  sc.va = reinterpret_cast<uint32_t*>(base + 4 * cap);
  sc.vb = sc.va + cap;
  sc.hist = sc.vb + cap;
  return sc;
}

template <int N>
__device__ __forceinline__ u64 morton_code(const int64_t* B) {
  u64 code = 0;
  constexpr int kb = key_bits(N) < 10 ? key_bits(N) : 10;  // 10 bits per coordinate suffice (|B| < 512)
#pragma unroll
  for (int bit = 0; bit < kb; ++bit)
#pragma unroll
    for (int j = 0; j < N; ++j) code |= static_cast<u64>(((B[j] + 512) >> bit) & 1) << (bit * N + j);
  return code;
}

// Sort keys of all bricks in [0, nb_prev): Morton code of survivors, ~0 for removed bricks.
template <int N, typename Real>
__global__ __launch_bounds__(kWG) void k_sort_keys(Dev<Real> d, int gate) {
  if (!gate_open(d, gate)) return;
  const SortScratch sc = sort_scratch(d);
  const uint32_t nb = min(d.sb->nb_prev, d.cap_b);
  uint32_t kept = 0;
  for (uint32_t b = blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += gridDim.x * blockDim.x) {
    int64_t B[N];
    unpack_key<N>(d.key[b], B);
    const bool alive = d.mask[b] != 0ull;
    sc.ka[b] = alive ? morton_code<N>(B) : ~0ull;
    sc.va[b] = b;
    kept += alive ? 1u : 0u;
  }
  for (int o = 32; o > 0; o >>= 1) kept += __shfl_xor(kept, o);
  if (lane_id() == 0 && kept) atomicAdd(&d.sb->nb_new, kept);
}

// Per-chunk histogram of digit `shift`.
template <typename Real>
__global__ __launch_bounds__(kWG) void k_sort_hist(Dev<Real> d, int gate, int shift, int flip) {
  if (!gate_open(d, gate)) return;
  const SortScratch sc = sort_scratch(d);
  const u64* keys = flip ? sc.kb : sc.ka;
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  uint64_t lo, hi;
  wg_chunk(min(d.sb->nb_prev, d.cap_b), lo, hi);
  for (uint64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
  __syncthreads();
  sc.hist[threadIdx.x * kSortWG + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of the digit-major histogram (256 x kSortWG entries).
// Inclusive prefix sum over the wave (lane l gets the sum of lanes 0..l).
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, int lane) {
#pragma unroll
  for (int o = 1; o < kLanes; o <<= 1) {
    const uint32_t u = static_cast<uint32_t>(__shfl_up(static_cast<int>(v), o));
    v += lane >= o ? u : 0u;
  }
  return v;
}

// Offsets of the radix scatter: digit-major exclusive prefix of the histogram
// (digit d, chunk w) -> sum over digits below d of their totals plus the
// counts of digit d in chunks below w.  One workgroup of 16 waves; each wave
// owns 16 digit rows, four chunks per lane (coalesced).  All of a wave's rows
// are loaded before any is used, so the kernel waits for memory about once
// rather than once per row.
constexpr int kScanWG = 1024;
constexpr int kScanRows = 256 / (kScanWG / kLanes);  // digit rows per wave
template <typename Real>
__global__ __launch_bounds__(kScanWG) void k_sort_scan(Dev<Real> d, int gate) {
  static_assert(kSortWG == 4 * kLanes, "four chunks per lane");
  if (!gate_open(d, gate)) return;
  const SortScratch sc = sort_scratch(d);
  __shared__ uint32_t tot[256];
  const int lane = lane_id(), w = threadIdx.x >> 6;
  constexpr int kWaves = kScanWG / kLanes;
  uint32_t v[kScanRows][4];
#pragma unroll
  for (int r = 0; r < kScanRows; ++r) {
    const uint32_t* row = sc.hist + static_cast<size_t>(w + kWaves * r) * kSortWG + 4 * lane;
#pragma unroll
    for (int q = 0; q < 4; ++q) v[r][q] = row[q];
  }
  uint32_t ex[kScanRows];  // exclusive prefix of this lane's chunks within the row
#pragma unroll
  for (int r = 0; r < kScanRows; ++r) {
    const uint32_t sum = v[r][0] + v[r][1] + v[r][2] + v[r][3];
    const uint32_t inc = wave_incl_scan(sum, lane);
    ex[r] = inc - sum;
    if (lane == kLanes - 1) tot[w + kWaves * r] = inc;
  }
  __syncthreads();
  if (w == 0) {
    const uint32_t a = tot[4 * lane], b = tot[4 * lane + 1], c = tot[4 * lane + 2], e = tot[4 * lane + 3];
    const uint32_t sum = a + b + c + e;
    const uint32_t x = wave_incl_scan(sum, lane) - sum;
    tot[4 * lane] = x;
    tot[4 * lane + 1] = x + a;
    tot[4 * lane + 2] = x + a + b;
    tot[4 * lane + 3] = x + a + b + c;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kScanRows; ++r) {
    const int dg = w + kWaves * r;
    uint32_t* row = sc.hist + static_cast<size_t>(dg) * kSortWG + 4 * lane;
    const uint32_t x = ex[r] + tot[dg];
    row[0] = x;
    row[1] = x + v[r][0];
    row[2] = x + v[r][0] + v[r][1];
    row[3] = x + v[r][0] + v[r][1] + v[r][2];
  }
}

// Stable scatter: elements of a chunk keep their order within each digit.
template <typename Real>
__global__ __launch_bounds__(kWG) void k_sort_scatter(Dev<Real> d, int gate, int shift, int flip) {
  if (!gate_open(d, gate)) return;
  const SortScratch sc = sort_scratch(d);
  const u64* kin = flip ? sc.kb : sc.ka;
  u64* kout = flip ? sc.ka : sc.kb;
  const uint32_t* vin = flip ? sc.vb : sc.va;
  uint32_t* vout = flip ? sc.va : sc.vb;
  __shared__ uint32_t base[256];
  __shared__ uint32_t cnt[kWavesPerWG][256];
  const int lane = lane_id(), w = threadIdx.x >> 6;
  base[threadIdx.x] = sc.hist[threadIdx.x * kSortWG + blockIdx.x];
  uint64_t lo, hi;
  wg_chunk(min(d.sb->nb_prev, d.cap_b), lo, hi);
  for (uint64_t r0 = lo; r0 < hi; r0 += kWG) {
    for (int k = 0; k < kWavesPerWG; ++k) cnt[k][threadIdx.x] = 0;
    __syncthreads();
    const uint64_t i = r0 + threadIdx.x;
    const bool valid = i < hi;
    const u64 key = valid ? kin[i] : 0ull;
    const uint32_t dig = static_cast<uint32_t>((key >> shift) & 255u);
    // lanes of this wave holding the same digit (multisplit by 8 ballots)
    u64 same = ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const u64 bb = ballot(((dig >> bit) & 1u) != 0u);
      same &= ((dig >> bit) & 1u) ? bb : ~bb;
    }
    const uint32_t rank = static_cast<uint32_t>(__popcll(same & ((1ull << lane) - 1ull)));
    const bool leader = valid && rank == 0;
    if (leader) cnt[w][dig] = static_cast<uint32_t>(__popcll(same));
    __syncthreads();
    if (valid) {
      uint32_t before = base[dig];
      for (int k = 0; k < w; ++k) before += cnt[k][dig];
      const uint32_t dst = before + rank;
      kout[dst] = key;
      vout[dst] = vin[i];
    }
    __syncthreads();
    uint32_t add = 0;
    for (int k = 0; k < kWavesPerWG; ++k) add += cnt[k][threadIdx.x];
    base[threadIdx.x] += add;
    __syncthreads();
  }
}

// Gather the survivors in sorted order: key/mask into scratch copies, densities
// into the other buffer with removed lanes cleared.
template <typename Real>
__global__ __launch_bounds__(kWG) void k_sort_permute(Dev<Real> d, int gate, int flip) {
  if (!gate_open(d, gate)) return;
  const SortScratch sc = sort_scratch(d);
  const uint32_t* perm = flip ? sc.vb : sc.va;  // result of the last pass
  const uint32_t nb_new = min(d.sb->nb_new, d.cap_b);
  const Real* P = cur_p(d);
  Real* Pn = next_p(d);
  const int lane = lane_id();
  const WaveRange rg = wave_range(nb_new);
  for (uint32_t k = rg.begin; k < rg.end; k += rg.step) {
    const uint32_t src = perm[k];
    const u64 m = d.mask[src];
    if (lane == 0) {
      sc.key2[k] = d.key[src];
      sc.mask2[k] = m;
    }
    const Real v = P[static_cast<size_t>(src) * kLanes + lane];
    Pn[static_cast<size_t>(k) * kLanes + lane] = ((m >> lane) & 1ull) ? v : Real(0);
  }
}

template <typename Real>
__global__ __launch_bounds__(kWG) void k_compact_finish(Dev<Real> d) {
  if (!d.sb->prun) return;
  const uint32_t nb_new = min(d.sb->nb_new, d.cap_b), nb_prev = min(d.sb->nb_prev, d.cap_b);
  const SortScratch sc = sort_scratch(d);
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  const uint64_t tid = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x;
  for (uint64_t b = tid; b < nb_prev; b += stride) {
    const u64 m = b < nb_new ? sc.mask2[b] : 0ull;
    if (b < nb_new) d.key[b] = sc.key2[b];
    d.mask[b] = m;
    d.abv[b] = m;
    d.done[b] = 0ull;
  }
  const uint64_t lo = uint64_t(nb_new) * kLanes, hi = uint64_t(nb_prev) * kLanes;
  for (uint64_t i = lo + tid; i < hi; i += stride) {
    d.P0[i] = Real(0);
    d.P1[i] = Real(0);
  }
}

// ---------------------------------------------------------------------------
// Marginals: scratch hashtable keyed by the projected cell index
// ---------------------------------------------------------------------------
template <int N, typename Real>
__global__ __launch_bounds__(kWG) void k_marg_accumulate(Dev<Real> d, uint32_t dim_mask, uint64_t tmask) {
  u64* tkey = reinterpret_cast<u64*>(d.Q);
  double* tval = reinterpret_cast<double*>(tkey + tmask + 1);
  const Real* P = cur_p(d);
  const int lane = lane_id();
  int nm = 0;
  for (int j = 0; j < N; ++j) nm += (dim_mask >> j) & 1u;
  const int kb = 63 / (nm > 0 ? nm : 1);
  const int64_t bias = int64_t(1) << (kb - 1);
  const WaveRange rg = wave_range(nb_of(d));
  for (uint32_t b = rg.begin; b < rg.end; b += rg.step) {
    const u64 m = d.mask[b];
    if (!((m >> lane) & 1ull)) continue;
    int64_t B[N];
    unpack_key<N>(d.key[b], B);
    int32_t ii[N];
    double xc[N];
    cell_of<N>(d, B, lane, ii, xc);
    u64 key = 0;
    int c = 0;
    for (int j = 0; j < N; ++j)
      if ((dim_mask >> j) & 1u) {
        key |= static_cast<u64>(static_cast<int64_t>(ii[j]) + bias) << (kb * c);
        ++c;
      }
    u64 h = mix64(key) & tmask;
    for (uint64_t probe = 0; probe <= tmask; ++probe) {
      u64 k = __hip_atomic_load(&tkey[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (k == kEmptyKey) {
        u64 expect = kEmptyKey;
        if (__hip_atomic_compare_exchange_strong(&tkey[h], &expect, key, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT))
          k = key;
        else
          k = expect;
      }
      if (k == key) {
        atomicAdd(&tval[h], static_cast<double>(P[static_cast<size_t>(b) * kLanes + lane]));
        break;
      }
      h = (h + 1) & tmask;
      if (probe == tmask) atomicOr(&d.sb->overflow, 1u);
    }
  }
}

template <typename Real>
__global__ void k_fill_marg(Dev<Real> d, uint64_t tmask) {
  u64* tkey = reinterpret_cast<u64*>(d.Q);
  double* tval = reinterpret_cast<double*>(tkey + tmask + 1);
  for (uint64_t i = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x; i <= tmask; i += uint64_t(gridDim.x) * blockDim.x) {
    tkey[i] = kEmptyKey;
    tval[i] = 0.0;
  }
}

// Compact the occupied table slots to the front: keys to tkey2[0, count), sums to tval2.
template <typename Real>
__global__ void k_marg_compact(Dev<Real> d, uint64_t tmask) {
  u64* tkey = reinterpret_cast<u64*>(d.Q);
  double* tval = reinterpret_cast<double*>(tkey + tmask + 1);
  u64* okey = reinterpret_cast<u64*>(tval + tmask + 1);
  double* oval = reinterpret_cast<double*>(okey + tmask + 1);
  for (uint64_t i = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x; i <= tmask; i += uint64_t(gridDim.x) * blockDim.x) {
    if (tkey[i] == kEmptyKey) continue;
    const uint32_t k = atomicAdd(&d.sb->nb_new, 1u);
    okey[k] = tkey[i];
    oval[k] = tval[i];
  }
}

// ---------------------------------------------------------------------------
// Probe statistics (Sec. 4.2): successful lookups of every brick key and
// unsuccessful lookups of keys that are not in the table.
// ---------------------------------------------------------------------------
template <typename Real>
__global__ void k_probe(Dev<Real> d, uint64_t n_miss, double* out) {
  const uint32_t nb = nb_of(d);
  double hit = 0.0, miss = 0.0;
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t i = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x; i < nb + n_miss; i += stride) {
    const u64 key = i < nb ? d.key[i] : (mix64(i * 0x9e3779b97f4a7c15ull + 12345ull) >> 1);
    u64 h = mix64(key) & d.hmask;
    double probes = 1.0;
    for (uint64_t p = 0; p <= d.hmask; ++p) {
      const u64 k = d.hkey[h];
      if (k == key || k == kEmptyKey) break;
      h = (h + 1) & d.hmask;
      probes += 1.0;
    }
    if (i < nb)
      hit += probes;
    else
      miss += probes;
  }
  hit = wave_sum(hit);
  miss = wave_sum(miss);
  if (lane_id() == 0) {
    atomicAdd(&out[0], hit);
    atomicAdd(&out[1], miss);
  }
}

// ---------------------------------------------------------------------------
// Launch sequences
// ---------------------------------------------------------------------------
template <int N, int MODEL, typename Real>
struct Ops {
  static const Dev<Real>& D(const void* p) { return *static_cast<const Dev<Real>*>(p); }

  // Survivors sorted by Morton code (prune gate); result in the sort scratch.
  static void reorder(const Dev<Real>& d, hipStream_t s, uint32_t G) {
    k_sort_keys<N, Real><<<G, kWG, 0, s>>>(d, kGatePrune);
    int flip = 0;
    for (int shift = 0; shift < 64; shift += 8, flip ^= 1) {
      k_sort_hist<Real><<<kSortWG, kWG, 0, s>>>(d, kGatePrune, shift, flip);
      k_sort_scan<Real><<<1, kScanWG, 0, s>>>(d, kGatePrune);
      k_sort_scatter<Real><<<kSortWG, kWG, 0, s>>>(d, kGatePrune, shift, flip);
    }
    k_sort_permute<Real><<<G, kWG, 0, s>>>(d, kGatePrune, flip);
  }

  static void rebuild_links(const Dev<Real>& d, hipStream_t s, uint32_t G, int gate) {
    k_hash_clear<Real><<<G, kWG, 0, s>>>(d, gate);
    k_hash_insert_all<Real><<<G, kWG, 0, s>>>(d, gate);
    k_relink_all<N, Real><<<G, kWG, 0, s>>>(d, gate);
  }

  static void normalise_gated(const Dev<Real>& d, hipStream_t s, uint32_t G, int gate) {
    k_reduce<N, Real><<<G, kWG, 0, s>>>(d, gate);
    k_final_reduce<Real><<<1, kWG, 0, s>>>(d, G, gate, 0);
    k_scale<N, Real><<<G, kWG, 0, s>>>(d, gate);
    k_final_reduce<Real><<<1, kWG, 0, s>>>(d, G, gate, 2);
  }

  static void init_gaussian(const void* p, hipStream_t s, uint32_t G, uint32_t Gbox) {
    const Dev<Real>& d = D(p);
    k_init_count<N, Real><<<Gbox, kWG, 0, s>>>(d);
    k_scan<<<1, kWG, 0, s>>>(d.part, Gbox, d.sb, kGateAlways, &d.sb->nb, d.cap_b);
    k_init_write<N, Real><<<Gbox, kWG, 0, s>>>(d);
    rebuild_links(d, s, G, kGateAlways);
    k_scalar<Real><<<1, 64, 0, s>>>(d, kOpResetSmax, 0.0);
    k_smax_all<N, MODEL, Real><<<G, kWG, 0, s>>>(d);
    normalise_gated(d, s, G, kGateAlways);
  }

  static void init_finish(const void* p, hipStream_t s, uint32_t G) {
    const Dev<Real>& d = D(p);
    rebuild_links(d, s, G, kGateAlways);
    k_scalar<Real><<<1, 64, 0, s>>>(d, kOpResetSmax, 0.0);
    k_smax_all<N, MODEL, Real><<<G, kWG, 0, s>>>(d);
    k_reduce<N, Real><<<G, kWG, 0, s>>>(d, kGateAlways);
    k_final_reduce<Real><<<1, kWG, 0, s>>>(d, G, kGateAlways, 2);
  }

  static void step(const void* p, hipStream_t s, uint32_t G, Profiler* pf) {
    const Dev<Real>& d = D(p);
    k_scalar<Real><<<1, 64, 0, s>>>(d, kOpStepBegin, 0.0);
    pf->begin(kProfGrow, s);
    if (d.grow_mode == 2)
      k_grow_orthant<N, MODEL, Real><<<G, kWG, 0, s>>>(d);
    else
      k_grow<N, MODEL, Real><<<G, kWG, 0, s>>>(d);
    pf->end(s);
    pf->begin(kProfGrowFix, s);
    k_grow_fix<N, MODEL, Real><<<G, kWG, 0, s>>>(d);
    pf->end(s);
    k_scalar<Real><<<1, 64, 0, s>>>(d, kOpDt, 0.0);
    pf->begin(kProfFluxA, s);
    k_flux_a<N, MODEL, Real><<<G, kWG, 0, s>>>(d);
    pf->end(s);
    pf->begin(kProfFluxB, s);
    k_flux_b<N, MODEL, Real><<<G, kWG, 0, s>>>(d);
    pf->end(s);
    k_final_step<Real><<<1, kWG, 0, s>>>(d, G);
  }

  static void step_multi(const MultiGrids& m, hipStream_t s) {
    if (m.R == 0) return;
    const uint32_t W = m.wg0[m.R];
    k_scalar_multi<Real><<<m.R, 64, 0, s>>>(m, kOpStepBegin);
    k_grow_multi<N, MODEL, Real><<<W, kWG, 0, s>>>(m);
    k_grow_fix_multi<N, MODEL, Real><<<W, kWG, 0, s>>>(m);
    k_scalar_multi<Real><<<m.R, 64, 0, s>>>(m, kOpDt);
    k_flux_a_multi<N, MODEL, Real><<<W, kWG, 0, s>>>(m);
    k_flux_b_multi<N, MODEL, Real><<<W, kWG, 0, s>>>(m);
    k_final_step_multi<Real><<<m.R, kWG, 0, s>>>(m);
  }

  static void prune(const void* p, hipStream_t s, uint32_t G, bool from_step, Profiler* pf) {
    const Dev<Real>& d = D(p);
    pf->begin(kProfPrune, s);
    k_scalar<Real><<<1, 64, 0, s>>>(d, from_step ? kOpPruneBeginStep : kOpPruneBeginAlways, 0.0);
    k_prune_above<N, Real><<<G, kWG, 0, s>>>(d);
    if (d.grow_mode == 2)
      k_prune_mark_orthant<N, MODEL, Real><<<G, kWG, 0, s>>>(d);
    else
      k_prune_mark<N, MODEL, Real><<<G, kWG, 0, s>>>(d);
    reorder(d, s, G);
    k_compact_finish<Real><<<G, kWG, 0, s>>>(d);
    k_scalar<Real><<<1, 64, 0, s>>>(d, kOpPruneCommit, 0.0);
    rebuild_links(d, s, G, kGatePrune);
    normalise_gated(d, s, G, kGatePrune);
    k_scalar<Real><<<1, 64, 0, s>>>(d, kOpPruneAccount, 0.0);
    pf->end(s);
  }

  static void correct(const void* p, hipStream_t s, uint32_t G, int comp, double y, double sigma, bool do_prune) {
    const Dev<Real>& d = D(p);
    k_correct<N, Real><<<G, kWG, 0, s>>>(d, comp, y, sigma);
    k_final_reduce<Real><<<1, kWG, 0, s>>>(d, G, kGateAlways, 2);
    if (do_prune) {
      Profiler none;
      prune(p, s, G, false, &none);
    } else {
      normalise_gated(d, s, G, kGateAlways);
    }
  }

  static void normalise(const void* p, hipStream_t s, uint32_t G, int gate) { normalise_gated(D(p), s, G, gate); }

  static void rollback(const void* p, hipStream_t s, uint32_t G) {
    const Dev<Real>& d = D(p);
    k_rollback<Real><<<G, kWG, 0, s>>>(d);
    k_scalar<Real><<<1, 64, 0, s>>>(d, kOpRollback, 0.0);
    rebuild_links(d, s, G, kGateAlways);
  }

  static void relink(const void* p, hipStream_t s, uint32_t G) { rebuild_links(D(p), s, G, kGateAlways); }

  static void set_tstop(const void* p, hipStream_t s, double t_stop) {
    k_scalar<Real><<<1, 64, 0, s>>>(D(p), kOpSetTStop, t_stop);
  }

  static void marginals(const void* p, hipStream_t s, uint32_t G, uint32_t dim_mask, uint64_t tmask) {
    const Dev<Real>& d = D(p);
    k_scalar<Real><<<1, 64, 0, s>>>(d, kOpMargBegin, 0.0);
    k_fill_marg<Real><<<G, kWG, 0, s>>>(d, tmask);
    k_marg_accumulate<N, Real><<<G, kWG, 0, s>>>(d, dim_mask, tmask);
    k_marg_compact<Real><<<G, kWG, 0, s>>>(d, tmask);
  }

  static void probe(const void* p, hipStream_t s, uint32_t G, uint64_t n_miss, double* out2) {
    k_probe<Real><<<G, kWG, 0, s>>>(D(p), n_miss, out2);
  }

  static const KernelTable* table(int prec) {
    static const KernelTable t = {N,          MODEL,   prec,      &init_gaussian, &init_finish, &step,
                                  &prune,     &correct, &normalise, &set_tstop,     &marginals,   &probe,
                                  &step_multi, &rollback, &relink};
    return &t;
  }
};

}  // namespace gbees
