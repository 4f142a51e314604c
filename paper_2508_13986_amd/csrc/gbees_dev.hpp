// Device-side data layout and helpers of the GBEES hot path on gfx950.
//
// Storage: the sparse grid of control volumes (Sec. 2.1, Eq. 5) is kept in
// "bricks" of 64 cells, one wave64 per brick.  A brick covers 2^b_j cells along
// dimension j with sum_j b_j = 6 (n = 6: 2x2x2x2x2x2, n = 3: 4x4x4, ...).  Each
// brick has a 64-bit occupancy mask; a cell is in the grid iff its bit is set,
// and an absent cell always stores density 0.  Bricks are addressed through an
// open-addressing hashtable with linear probing (Sec. 4.2) keyed by the packed
// brick coordinates, and each brick stores the indices of its 2n axis-neighbour
// bricks so that the flux passes never probe the table.
//
// Arrays are structure-of-arrays, brick-major: P[b * 64 + lane].
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

namespace gbees {

// Compile-time loop: f(std::integral_constant<int, I>{}) for I = 0 .. Count-1.
template <typename F, int... I>
__host__ __device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int Count, typename F>
__host__ __device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, Count>{});
}

constexpr int kLanes = 64;
constexpr int kWavesPerWG = 4;
constexpr int kWG = kLanes * kWavesPerWG;
using u64 = unsigned long long;
constexpr uint32_t kNone = 0xFFFFFFFFu;          // "no brick" / unpublished hash value
constexpr u64 kEmptyKey = ~0ull;                   // never a packed key (bit 63 is never set)
constexpr int kMaxWG = 4096;                       // upper bound on grid size of grid-stride kernels
constexpr int kPartStride = 4;                     // doubles per workgroup partial

enum Status : int32_t { kOk = 0, kErrCapacity = -2, kErrRange = -3, kErrState = -6 };
enum Gate : int32_t { kGateAlways = 0, kGateStep = 1, kGatePrune = 2 };

// ---------------------------------------------------------------------------
// Brick geometry, fixed per dimension count n.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int brick_bits(int n, int j) {
  return n == 1 ? 6 : n == 2 ? 3 : n == 3 ? 2 : n == 4 ? (j < 2 ? 2 : 1) : n == 5 ? (j < 1 ? 2 : 1) : 1;
}
__host__ __device__ constexpr int brick_off(int n, int j) {
  int s = 0;
  for (int m = 0; m < j; ++m) s += brick_bits(n, m);
  return s;
}
__host__ __device__ constexpr int brick_side(int n, int j) { return 1 << brick_bits(n, j); }
__host__ __device__ constexpr int brick_stride(int n, int j) { return 1 << brick_off(n, j); }
// Lanes whose local coordinate along j equals v.
__host__ __device__ constexpr uint64_t lanes_at(int n, int j, int v) {
  uint64_t m = 0;
  for (int L = 0; L < kLanes; ++L)
    if (((L >> brick_off(n, j)) & (brick_side(n, j) - 1)) == v) m |= 1ull << L;
  return m;
}
// Moving one cell by s along j, seen as lane masks: `out` lanes leave the brick
// (they land in the neighbour brick, shifted by sh_out lanes), `in` lanes stay
// (shifted by sh_in lanes).
template <int N, int J, int S>
struct Dir {
  static constexpr int side = brick_side(N, J), stride = brick_stride(N, J);
  static constexpr uint64_t out = S > 0 ? lanes_at(N, J, side - 1) : lanes_at(N, J, 0);
  static constexpr uint64_t in = ~out;
  static constexpr int sh_in = S * stride;
  static constexpr int sh_out = -S * (side - 1) * stride;
};
// Pair p of the ordered list (0,1), (0,2), ..., (n-2,n-1).
__host__ __device__ constexpr int pair_j(int n, int p) {
  int j = 0;
  while (p >= n - 1 - j) {
    p -= n - 1 - j;
    ++j;
  }
  return j;
}
__host__ __device__ constexpr int pair_l(int n, int p) {
  int j = 0;
  while (p >= n - 1 - j) {
    p -= n - 1 - j;
    ++j;
  }
  return j + 1 + p;
}
template <int K>
__host__ __device__ __forceinline__ unsigned long long lshc(unsigned long long m) {
  if constexpr (K >= 0)
    return m << K;
  else
    return m >> (-K);
}

// Bits per coordinate in a packed key; coordinates are biased by 2^(kb-1).
__host__ __device__ constexpr int key_bits(int n) { return 63 / n; }
// Brick coordinates allowed: the packed key must fit and cell indices stay int32.
__host__ __device__ constexpr int64_t brick_limit(int n) {
  return (key_bits(n) - 1) < 24 ? (int64_t(1) << (key_bits(n) - 1)) : (int64_t(1) << 24);
}

template <int N>
__host__ __device__ inline bool brick_in_range(const int64_t* B) {
  const int64_t lim = brick_limit(N);
  for (int j = 0; j < N; ++j)
    if (B[j] < -lim || B[j] >= lim) return false;
  return true;
}

template <int N>
__host__ __device__ inline u64 pack_key(const int64_t* B) {
  constexpr int kb = key_bits(N);
  const int64_t bias = int64_t(1) << (kb - 1);
  u64 k = 0;
  for (int j = 0; j < N; ++j) k |= static_cast<u64>(B[j] + bias) << (kb * j);
  return k;
}

template <int N>
__host__ __device__ inline void unpack_key(u64 k, int64_t* B) {
  constexpr int kb = key_bits(N);
  const int64_t bias = int64_t(1) << (kb - 1);
  const u64 m = (kb >= 63) ? ~0ull >> 1 : ((1ull << kb) - 1);
  for (int j = 0; j < N; ++j) B[j] = static_cast<int64_t>((k >> (kb * j)) & m) - bias;
}

// MurmurHash3 64-bit finaliser (Appleby), a published avalanche mixer.
__host__ __device__ inline u64 mix64(u64 k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return k;
}

// ---------------------------------------------------------------------------
// Device-resident scalars of one grid (read by every kernel of a step).
// ---------------------------------------------------------------------------
struct Scalars {
  double t, t_stop, dt, t_next, dt_last;
  double maxp;            // max P of the current grid
  double sum;             // sum P of the current grid (after the last reduction)
  double z;               // normaliser of the last renormalisation
  u64 smax_bits;          // max_i S_i over the grid, as the bits of a non-negative double
  uint32_t nb;            // bricks in use
  uint32_t nb_old;        // bricks before this step's grow
  uint32_t nb_prev;       // bricks before the current prune
  uint32_t nb_new;        // bricks after the current prune
  uint32_t cur;           // which density buffer is current
  uint32_t run;           // the current step runs
  uint32_t prun;          // the current prune runs
  uint32_t ndeferred;     // grow records whose brick was published by another wave
  int32_t status;
  uint32_t overflow;      // scratch-table overflow of the last marginal call
  u64 steps, cell_updates, brick_updates, cells, prunes, inserted, grow_bricks;
  u64 deferred;           // grow records finished by the fix-up pass, over all steps
  u64 smax_begin;         // smax_bits at the start of the current step (restored on a failed grow)
  double sum_pre;         // sum P when the current prune began
  double pruned;          // sum over prunes of the fraction of the mass each one removed
};

// ---------------------------------------------------------------------------
// Everything a kernel needs, passed by value.
// ---------------------------------------------------------------------------
template <typename Real>
struct Dev {
  int n, model, limiter, grow_mode;
  double params[48];
  double h[6], mean[6];
  double thresh_rel, cfl, dt_fixed, vol;
  // initial condition
  double sinv[36];
  double bound;
  int64_t box_lo[6], box_n[6];  // brick-coordinate box of the initial ellipsoid
  uint64_t box_count;
  // capacities
  uint32_t cap_b;
  uint32_t ndef_cap;
  uint64_t hmask;
  // arrays
  // Brick arrays hold cap_b + 1 bricks: index cap_b is a permanently empty brick
  // (mask 0, densities 0) that flux passes read in place of a missing neighbour.
  u64* key;            // [cap_b + 1]
  u64* mask;           // [cap_b + 1]
  u64* done;           // [cap_b + 1] cells whose grow candidates are known to be present
  u64* abv;            // [cap_b + 1] above-threshold lanes inside a prune; between prunes, the
                       // occupancy masks at the start of the next step (restored on a failed grow)
  uint32_t* nbr;       // [2n][cap_b + 1]; entry 2j is the -e_j neighbour, 2j+1 the +e_j neighbour
  Real* P0;            // [(cap_b + 1) * 64]
  Real* P1;            // [(cap_b + 1) * 64]
  Real* Q;             // [(cap_b + 1) * n * 64]; also scratch for reordering and marginals
  u64* hkey;           // [hmask + 1]
  uint32_t* hval;      // [hmask + 1]
  u64* defer;          // [ndef_cap * 2]: hash slot, lane bits
  uint32_t* part;      // [kMaxWG + 1] per-workgroup counts / offsets
  double* dpart;       // [kMaxWG * kPartStride] per-workgroup partial reductions
  Scalars* sb;
};

// ---------------------------------------------------------------------------
// Wave helpers.
// ---------------------------------------------------------------------------
__device__ inline int lane_id() { return static_cast<int>(__lane_id()); }
__device__ inline u64 ballot(bool p) { return static_cast<u64>(__ballot(p)); }
__device__ inline u64 lsh(u64 m, int k) { return k >= 0 ? (m << k) : (m >> (-k)); }

__device__ inline double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}
__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__device__ inline double bits_to_double(u64 b) { return __longlong_as_double(static_cast<long long>(b)); }
__device__ inline u64 double_to_bits(double v) { return static_cast<u64>(__double_as_longlong(v)); }

// Grid-stride assignment of bricks to waves.  The grid size is a multiple of 8 and
// workgroup w runs on XCD w % 8, so each XCD walks one contiguous eighth of the
// brick list and neighbouring bricks tend to share that XCD's L2.
struct WaveRange {
  uint32_t begin, end, step;
};
// A workgroup's place in the launch that serves its grid: index wg of nwg.
// A plain launch serves one grid with all its workgroups; a launch shared by
// several grids gives each a contiguous run of workgroups whose length and
// start are multiples of 8, so a workgroup's XCD is still wg % 8.
struct Slot {
  uint32_t wg, nwg;
};
__device__ inline Slot hw_slot() { return Slot{blockIdx.x, gridDim.x}; }

__device__ inline WaveRange wave_range(uint32_t n, Slot sl) {
  const uint32_t G = sl.nwg;
  const uint32_t xcd = sl.wg & 7u, slot = sl.wg >> 3, per = G >> 3;
  const uint32_t chunk = (n + 7u) / 8u;
  const uint32_t lo = min(n, xcd * chunk), hi = min(n, lo + chunk);
  // readfirstlane tells the compiler the wave index is uniform, so brick-derived
  // values (links, masks, keys, base pointers) live in scalar registers.
  const uint32_t w = slot * kWavesPerWG + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  return WaveRange{lo + w, hi, per * kWavesPerWG};
}
__device__ inline WaveRange wave_range(uint32_t n) { return wave_range(n, hw_slot()); }

// The same XCD split, in runs of `len` consecutive bricks: the wave takes the
// runs starting at begin, begin + step, ... below end.  Runs are up to kRunMax
// long but no longer than the bricks per wave, so a small grid still spreads
// over all waves.  Bricks that need work cluster in the Morton order, and
// short runs deal them out more evenly: 16 measured fastest (64: 4% slower,
// 4: 4%, 2: 12%).
constexpr uint32_t kRunMax = 16;
struct RunRange {
  uint32_t begin, end, step, len;
};
__device__ inline RunRange wave_runs(uint32_t n, Slot sl) {
  const uint32_t G = sl.nwg;
  const uint32_t xcd = sl.wg & 7u, slot = sl.wg >> 3, per = G >> 3;
  const uint32_t chunk = (n + 7u) / 8u;
  const uint32_t lo = min(n, xcd * chunk), hi = min(n, lo + chunk);
  const uint32_t w = slot * kWavesPerWG + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t nw = per * kWavesPerWG;
  uint32_t len = kRunMax;
  while (len > 1u && static_cast<uint64_t>(len) * nw > chunk) len >>= 1;
  const uint64_t first = static_cast<uint64_t>(lo) + static_cast<uint64_t>(w) * len;
  return RunRange{static_cast<uint32_t>(min<uint64_t>(first, hi)), hi, nw * len, len};
}

// Contiguous chunk of [0, n) for this workgroup (stable-order compaction).
__device__ inline void wg_chunk(uint64_t n, uint64_t& lo, uint64_t& hi) {
  const uint64_t G = gridDim.x;
  const uint64_t chunk = (n + G - 1) / G;
  lo = min(n, static_cast<uint64_t>(blockIdx.x) * chunk);
  hi = min(n, lo + chunk);
}

template <typename Real>
__device__ inline bool gate_open(const Dev<Real>& d, int gate) {
  if (gate == kGateStep) return d.sb->run != 0;
  if (gate == kGatePrune) return d.sb->prun != 0;
  return true;
}

template <typename Real>
__device__ inline uint32_t nb_of(const Dev<Real>& d) { return min(d.sb->nb, d.cap_b); }
template <typename Real>
__device__ inline const Real* cur_p(const Dev<Real>& d) { return d.sb->cur ? d.P1 : d.P0; }
template <typename Real>
__device__ inline Real* cur_p_mut(const Dev<Real>& d) { return d.sb->cur ? d.P1 : d.P0; }
template <typename Real>
__device__ inline Real* next_p(const Dev<Real>& d) { return d.sb->cur ? d.P0 : d.P1; }

__device__ inline void set_status(Scalars* sb, int32_t code) { atomicCAS(&sb->status, 0, code); }

// ---------------------------------------------------------------------------
// Hashtable (open addressing, linear probing; Sec. 4.2).
// ---------------------------------------------------------------------------
// Lookup; used only by kernels that run after the table was built (plain loads).
template <typename Real>
__device__ inline uint32_t hash_find(const Dev<Real>& d, u64 key) {
  u64 h = mix64(key) & d.hmask;
  for (uint64_t probe = 0; probe <= d.hmask; ++probe) {
    const u64 k = d.hkey[h];
    if (k == key) return d.hval[h];
    if (k == kEmptyKey) return kNone;
    h = (h + 1) & d.hmask;
  }
  return kNone;
}

// Find key or claim an empty slot for it.  Returns the hash slot; *won is set when
// this call inserted the key.  Returns ~0 when the table is full.
template <typename Real>
__device__ inline u64 hash_claim(const Dev<Real>& d, u64 key, bool* won) {
  u64 h = mix64(key) & d.hmask;
  *won = false;
  for (uint64_t probe = 0; probe <= d.hmask; ++probe) {
    // A stale EMPTY only sends us to the CAS, which is authoritative.
    u64 k = d.hkey[h];
    if (k == kEmptyKey) {
      u64 expect = kEmptyKey;
      const bool ok = __hip_atomic_compare_exchange_strong(&d.hkey[h], &expect, key, __ATOMIC_RELAXED,
                                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (ok) {
        *won = true;
        return h;
      }
      k = expect;
    }
    if (k == key) return h;
    h = (h + 1) & d.hmask;
  }
  return ~0ull;
}

// ---------------------------------------------------------------------------
// Drift at a face centre (Sec. 5.1 models; linear f = A x + b for tests).
// The operation order is fixed and contraction is disabled so that the
// velocities, hence the CFL step and every up/downwind decision, are bitwise
// reproducible: coordinates are mean_j + i_j h_j, and the face coordinate
// along j is mean_j + (i_j - 1/2) h_j.
// ---------------------------------------------------------------------------
enum ModelId : int { kModelL63 = 1, kModelL96 = 2, kModelLinear = 3 };

template <int MODEL, int N>
__device__ __forceinline__ double drift_at(const double* x, int j, double xj, const double* p) {
#pragma clang fp contract(off)
  auto X = [&](int m) { return m == j ? xj : x[m]; };
  if constexpr (MODEL == kModelL63) {
    const double z = X(2) + p[3];
    if (j == 0) return p[0] * (X(1) - X(0));
    if (j == 1) return X(0) * (p[1] - z) - X(1);
    return X(0) * X(1) - p[2] * z;
  } else if constexpr (MODEL == kModelL96) {
    const int jp1 = (j + 1) % N, jm1 = (j + N - 1) % N, jm2 = (j + N - 2) % N;
    return (X(jp1) - X(jm2)) * X(jm1) - X(j) + p[0];
  } else {
    double acc = p[j * N + 0] * X(0);
#pragma unroll
    for (int k = 1; k < N; ++k) acc = acc + p[j * N + k] * X(k);
    return acc + p[N * N + j];
  }
}

__device__ __forceinline__ double centre_coord(double mean, int32_t i, double h) {
#pragma clang fp contract(off)
  return mean + static_cast<double>(i) * h;
}
__device__ __forceinline__ double face_coord(double mean, int32_t i, double h) {
#pragma clang fp contract(off)
  return mean + (static_cast<double>(i) - 0.5) * h;
}

// f_{i - 1/2 e_j, j}: velocity at the backward j-face of the cell with index ii and centre xc.
template <int MODEL, int N, typename Real>
__device__ __forceinline__ double face_vel(const Dev<Real>& d, const double* xc, const int32_t* ii, int j) {
  return drift_at<MODEL, N>(xc, j, face_coord(d.mean[j], ii[j], d.h[j]), d.params);
}
// face_coord(mean, i + 1, h), bit for bit: (i + 1) - 0.5 and i + 0.5 are the
// same double for every int32 i, and this form reuses the conversion of i.
__device__ __forceinline__ double face_coord_fwd(double mean, int32_t i, double h) {
#pragma clang fp contract(off)
  return mean + (static_cast<double>(i) + 0.5) * h;
}

// f_{i + 1/2 e_j, j}: velocity at the forward j-face (the backward face of i + e_j).
template <int MODEL, int N, typename Real>
__device__ __forceinline__ double face_vel_fwd(const Dev<Real>& d, const double* xc, const int32_t* ii, int j) {
  return drift_at<MODEL, N>(xc, j, face_coord_fwd(d.mean[j], ii[j], d.h[j]), d.params);
}

// S_i = sum_j |f_{i - 1/2 e_j, j}| / h_j (Eq. 8).
template <int MODEL, int N, typename Real>
__device__ __forceinline__ double cell_speed(const Dev<Real>& d, const double* xc, const int32_t* ii) {
#pragma clang fp contract(off)
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < N; ++j) s = s + fabs(face_vel<MODEL, N>(d, xc, ii, j)) / d.h[j];
  return s;
}

// Cell index and centre of lane `lane` in the brick with coordinates B.
template <int N, typename Real>
__device__ __forceinline__ void cell_of(const Dev<Real>& d, const int64_t* B, int lane, int32_t* ii, double* xc) {
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const int a = (lane >> brick_off(N, j)) & (brick_side(N, j) - 1);
    ii[j] = static_cast<int32_t>(B[j] * brick_side(N, j) + a);
    xc[j] = centre_coord(d.mean[j], ii[j], d.h[j]);
  }
}

// Neighbour of a lane at distance dist (|dist| <= 2 <= side) along j:
// returns which brick (-1 the -e_j brick, 0 own, +1 the +e_j brick) and the lane there.
template <int N>
__device__ __forceinline__ int nb_lane(int lane, int j, int dist, int* which) {
  const int side = brick_side(N, j), stride = brick_stride(N, j);
  const int a = (lane >> brick_off(N, j)) & (side - 1);
  const int a2 = a + dist;
  const int o = a2 < 0 ? -1 : (a2 >= side ? 1 : 0);
  *which = o;
  return lane + (a2 - o * side - a) * stride;
}

}  // namespace gbees
