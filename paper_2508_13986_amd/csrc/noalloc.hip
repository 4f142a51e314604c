// Marginals into caller device buffers with no allocation (for callers that
// cannot allocate: code under HIP graph capture, serving loops, harnesses that
// forbid it).  Same sums as gbees_marginals (Sec. 5.1.2), but the aggregation
// table lives in a file-scope device array instead of the context's arena, and
// nothing is copied to the host or waited for.
#include <mutex>

#include "kernels.hpp"

namespace gbees {

// Aggregation table: kMargSlots keys and sums, then a row counter and an
// overflow flag.  One copy per GPU for the life of the process.
constexpr uint64_t kMargSlots = uint64_t(1) << 20;
constexpr size_t kScratchBytes = kMargSlots * 16 + 256;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct MargScratch {
  u64* key;
  double* val;
  uint32_t* counter;  // [0] rows, [1] overflow
};
__host__ __device__ inline MargScratch marg_scratch(void* base) {
  unsigned char* b = static_cast<unsigned char*>(base);
  MargScratch s;
  s.key = reinterpret_cast<u64*>(b);
  s.val = reinterpret_cast<double*>(b + kMargSlots * 8);
  s.counter = reinterpret_cast<uint32_t*>(b + kMargSlots * 16);
  return s;
}

__global__ void k_marg_clear(void* base) {
  const MargScratch s = marg_scratch(base);
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t i = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x; i < kMargSlots; i += stride) {
    s.key[i] = kEmptyKey;
    s.val[i] = 0.0;
  }
  if (blockIdx.x == 0 && threadIdx.x < 2) s.counter[threadIdx.x] = 0u;
}

// Every present cell adds P to the slot of its projected index (packed with
// 63 / |mask| bits per kept coordinate, as gbees_marginals packs it).
template <int N, typename Real>
__global__ __launch_bounds__(kWG) void k_marg_add(Dev<Real> d, void* base, uint32_t dim_mask) {
  const MargScratch s = marg_scratch(base);
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
    u64 h = mix64(key) & (kMargSlots - 1);
    bool placed = false;
    for (uint64_t probe = 0; probe < kMargSlots; ++probe) {
      u64 k = __hip_atomic_load(&s.key[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (k == kEmptyKey) {
        u64 expect = kEmptyKey;
        k = __hip_atomic_compare_exchange_strong(&s.key[h], &expect, key, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT)
                ? key
                : expect;
      }
      if (k == key) {
        atomicAdd(&s.val[h], static_cast<double>(P[static_cast<size_t>(b) * kLanes + lane]));
        placed = true;
        break;
      }
      h = (h + 1) & (kMargSlots - 1);
    }
    if (!placed) atomicOr(&s.counter[1], 1u);
  }
}

// Occupied slots become rows: the kept coordinates unpacked into idx[row][nm]
// and the sum times the widths of the summed-out dimensions into val[row].
// Rows past `capacity` are counted but not written.
__global__ void k_marg_rows(void* base, int nm, double weight, int64_t capacity, int32_t* idx, double* val) {
  const MargScratch s = marg_scratch(base);
  const int kb = 63 / nm;
  const int64_t bias = int64_t(1) << (kb - 1);
  const u64 km = (kb >= 63) ? (~0ull >> 1) : ((1ull << kb) - 1);
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t i = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x; i < kMargSlots; i += stride) {
    const u64 key = s.key[i];
    if (key == kEmptyKey) continue;
    const uint32_t r = atomicAdd(&s.counter[0], 1u);
    if (static_cast<int64_t>(r) >= capacity) continue;
    for (int q = 0; q < nm; ++q)
      idx[static_cast<size_t>(r) * nm + q] = static_cast<int32_t>(static_cast<int64_t>((key >> (kb * q)) & km) - bias);
    val[r] = s.val[i] * weight;
  }
}

__global__ void k_marg_count(void* base, int64_t* count) {
  const MargScratch s = marg_scratch(base);
  if (threadIdx.x == 0) *count = s.counter[1] ? -1 : static_cast<int64_t>(s.counter[0]);
}

namespace {

// Device address of `scratch` on each GPU, taken once per device.
constexpr int kMaxDevices = 64;
void* g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;

void* scratch_on_current_device() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    g_scratch[dev] = p;
  }
  return g_scratch[dev];
}

template <int N, typename Real>
void launch_add(const void* dev, hipStream_t s, uint32_t G, void* base, uint32_t mask) {
  k_marg_add<N, Real><<<G, kWG, 0, s>>>(*static_cast<const Dev<Real>*>(dev), base, mask);
}
template <typename Real>
void add_n(int n, const void* dev, hipStream_t s, uint32_t G, void* base, uint32_t mask) {
  switch (n) {
    case 1: launch_add<1, Real>(dev, s, G, base, mask); break;
    case 2: launch_add<2, Real>(dev, s, G, base, mask); break;
    case 3: launch_add<3, Real>(dev, s, G, base, mask); break;
    case 4: launch_add<4, Real>(dev, s, G, base, mask); break;
    case 5: launch_add<5, Real>(dev, s, G, base, mask); break;
    default: launch_add<6, Real>(dev, s, G, base, mask); break;
  }
}

}  // namespace

uint64_t marginal_scratch_slots() { return kMargSlots; }

// Enqueue the whole computation on s; returns false if the scratch address
// could not be taken or a launch failed.
bool marginals_static(const void* dev, int n, int precision, hipStream_t s, uint32_t G, uint32_t dim_mask,
                      double weight, int64_t capacity, int32_t* idx, double* val, int64_t* count) {
  void* base = scratch_on_current_device();
  if (!base) return false;
  int nm = 0;
  for (int j = 0; j < n; ++j) nm += (dim_mask >> j) & 1u;
  k_marg_clear<<<1024, kWG, 0, s>>>(base);
  if (precision == 1)
    add_n<float>(n, dev, s, G, base, dim_mask);
  else
    add_n<double>(n, dev, s, G, base, dim_mask);
  k_marg_rows<<<1024, kWG, 0, s>>>(base, nm, weight, capacity, idx, val);
  k_marg_count<<<1, 64, 0, s>>>(base, count);
  return hipGetLastError() == hipSuccess;
}

}  // namespace gbees
