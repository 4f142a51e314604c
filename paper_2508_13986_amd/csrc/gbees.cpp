// C ABI of the GBEES hot path (include/gbees.h): context, arena layout, the
// step driver, and the marshalling of exports.  All arithmetic of the method
// runs in the kernels of kernels.hip; host code here only validates inputs,
// lays out the caller's arena, enqueues launch sequences and copies results.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <cstring>
#include <new>
#include <unordered_map>
#include <vector>

#include "gbees.h"
#include "gbees_host.hpp"

using gbees::Dev;
using gbees::KernelTable;
using gbees::Scalars;
using gbees::u64;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  uint32_t cap_b = 0;
  u64 hcap = 0;
  uint32_t ndef = 0;
  size_t real_size = 8, qbytes = 0;
  size_t sb = 0, part = 0, dpart = 0, key = 0, mask = 0, done = 0, abv = 0, P0 = 0, P1 = 0;
  size_t zero_end = 0;
  size_t hkey = 0, hval = 0;
  size_t ff_end = 0;
  size_t nbr = 0, Q = 0, defer = 0;
  size_t devc = 0;  // device copy of the grid's Dev block (shared multi-grid launches read it)
  size_t total = 0;
};

int effective_model(const gbees_config& c) { return c.model == GBEES_UNIFORM ? GBEES_LINEAR : c.model; }

bool valid_config(const gbees_config& c) {
  if (c.n < 1 || c.n > 6) return false;
  if (c.model < GBEES_L63 || c.model > GBEES_UNIFORM) return false;
  if (!gbees::kernel_table(effective_model(c), c.n, c.precision == 1 ? 1 : 0)) return false;
  for (int j = 0; j < c.n; ++j)
    if (!(c.h[j] > 0.0) || !std::isfinite(c.h[j]) || !std::isfinite(c.mean[j])) return false;
  if (!(c.thresh_rel >= 0.0 && c.thresh_rel < 1.0)) return false;
  if (!(c.dt_fixed > 0.0) && !(c.cfl > 0.0 && c.cfl <= 1.0)) return false;
  if (c.prune_every < 0 || (c.limiter != 0 && c.limiter != 1) || c.grow_mode < 0 || c.grow_mode > 2) return false;
  if (c.precision != 0 && c.precision != 1) return false;
  if (c.max_cells < gbees::kLanes) return false;
  if (c.max_cells / gbees::kLanes > 0xF0000000ll) return false;
  return true;
}

bool make_layout(const gbees_config& c, Layout* L) {
  if (!valid_config(c)) return false;
  L->cap_b = static_cast<uint32_t>((c.max_cells + gbees::kLanes - 1) / gbees::kLanes);
  const double load = (c.hash_load > 0.0 && c.hash_load < 1.0) ? c.hash_load : 0.5;
  u64 want = static_cast<u64>(std::ceil(L->cap_b / load));
  u64 h = 1;
  while (h < want) h <<= 1;
  L->hcap = h;
  L->ndef = L->cap_b;
  L->real_size = c.precision == 1 ? 4 : 8;
  // Q also serves as scratch: the prune-time radix sort needs 48 B per brick plus
  // a 256 x 256 histogram; marginals need 32 B per table slot.
  L->qbytes = std::max((static_cast<size_t>(L->cap_b) + 1) * gbees::kLanes * std::max<size_t>(c.n * L->real_size, 32),
                       static_cast<size_t>(L->cap_b) * 48 + (size_t(1) << 20));
  const size_t cb = static_cast<size_t>(L->cap_b) + 1;  // + the permanently empty brick at index cap_b
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  L->sb = take(sizeof(Scalars));
  L->part = take((gbees::kMaxWG + 1) * sizeof(uint32_t));
  L->dpart = take(gbees::kMaxWG * gbees::kPartStride * sizeof(double));
  L->key = take(cb * 8);
  L->mask = take(cb * 8);
  L->done = take(cb * 8);
  L->abv = take(cb * 8);
  L->P0 = take(cb * gbees::kLanes * L->real_size);
  L->P1 = take(cb * gbees::kLanes * L->real_size);
  L->zero_end = o;
  L->hkey = take(L->hcap * 8);
  L->hval = take(L->hcap * 4);
  L->ff_end = o;
  L->nbr = take(2 * static_cast<size_t>(c.n) * cb * 4);
  L->Q = take(L->qbytes);
  L->defer = take(static_cast<size_t>(L->ndef) * 16);
  static_assert(sizeof(gbees::Dev<double>) == sizeof(gbees::Dev<float>), "one Dev slot for both precisions");
  L->devc = take(sizeof(gbees::Dev<double>));
  L->total = o;
  return true;
}

template <typename Real>
void fill_dev(Dev<Real>& d, const gbees_config& c, const Layout& L, char* base) {
  std::memset(&d, 0, sizeof(d));
  d.n = c.n;
  d.model = effective_model(c);
  d.limiter = c.limiter;
  d.grow_mode = c.grow_mode;
  if (c.model == GBEES_UNIFORM) {
    // f = b as the linear field with A = 0: 0 * x + ... + b_j == b_j exactly.
    for (int j = 0; j < c.n; ++j) d.params[c.n * c.n + j] = c.params[j];
  } else {
    std::memcpy(d.params, c.params, sizeof(d.params));
  }
  double vol = 1.0;
  for (int j = 0; j < c.n; ++j) {
    d.h[j] = c.h[j];
    d.mean[j] = c.mean[j];
    vol = vol * c.h[j];
  }
  d.vol = vol;
  d.thresh_rel = c.thresh_rel;
  d.cfl = c.cfl;
  d.dt_fixed = c.dt_fixed;
  d.cap_b = L.cap_b;
  d.ndef_cap = L.ndef;
  d.hmask = L.hcap - 1;
  d.sb = reinterpret_cast<Scalars*>(base + L.sb);
  d.part = reinterpret_cast<uint32_t*>(base + L.part);
  d.dpart = reinterpret_cast<double*>(base + L.dpart);
  d.key = reinterpret_cast<u64*>(base + L.key);
  d.mask = reinterpret_cast<u64*>(base + L.mask);
  d.done = reinterpret_cast<u64*>(base + L.done);
  d.abv = reinterpret_cast<u64*>(base + L.abv);
  d.P0 = reinterpret_cast<Real*>(base + L.P0);
  d.P1 = reinterpret_cast<Real*>(base + L.P1);
  d.hkey = reinterpret_cast<u64*>(base + L.hkey);
  d.hval = reinterpret_cast<uint32_t*>(base + L.hval);
  d.nbr = reinterpret_cast<uint32_t*>(base + L.nbr);
  d.Q = reinterpret_cast<Real*>(base + L.Q);
  d.defer = reinterpret_cast<u64*>(base + L.defer);
}

// Inverse of a symmetric positive definite matrix by Gauss-Jordan elimination
// with partial pivoting; false if singular or not positive definite.
bool spd_inverse(int n, const double* a_in, double* inv) {
  double a[6][12];
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < 2 * n; ++c) a[r][c] = c < n ? a_in[r * n + c] : (c - n == r ? 1.0 : 0.0);
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < r; ++c)
      if (a_in[r * n + c] != a_in[c * n + r]) return false;
  // positive definiteness via Cholesky pivots
  double l[6][6] = {};
  for (int j = 0; j < n; ++j) {
    double s = a_in[j * n + j];
    for (int k = 0; k < j; ++k) s -= l[j][k] * l[j][k];
    if (!(s > 0.0)) return false;
    l[j][j] = std::sqrt(s);
    for (int i = j + 1; i < n; ++i) {
      double t = a_in[i * n + j];
      for (int k = 0; k < j; ++k) t -= l[i][k] * l[j][k];
      l[i][j] = t / l[j][j];
    }
  }
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (std::fabs(a[r][col]) > std::fabs(a[piv][col])) piv = r;
    if (a[piv][col] == 0.0) return false;
    if (piv != col)
      for (int c = 0; c < 2 * n; ++c) std::swap(a[piv][c], a[col][c]);
    const double dv = a[col][col];
    for (int c = 0; c < 2 * n; ++c) a[col][c] = a[col][c] / dv;
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      const double f = a[r][col];
      if (f == 0.0) continue;
      for (int c = 0; c < 2 * n; ++c) a[r][c] = a[r][c] - f * a[col][c];
    }
  }
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < n; ++c) inv[r * n + c] = a[r][c + n];
  return true;
}

// Workgroups of a grid-stride launch over `bricks` bricks: about `per_wave`
// bricks per wave, but no fewer than 256 workgroups (or one per two waves'
// worth of bricks, if that is fewer), so that a small grid still spreads over
// the chip; a multiple of 8 (one run per XCD), at most kMaxWG.  Fewer, longer
// waves amortise each wave's start (its first loads are not overlapped) and
// leave room on the chip for other streams' launches.
uint32_t grid_for(uint64_t bricks, uint32_t per_wave) {
  const uint64_t per_wg = static_cast<uint64_t>(per_wave) * gbees::kWavesPerWG;
  const uint64_t fine = (bricks + 2 * gbees::kWavesPerWG - 1) / (2 * gbees::kWavesPerWG);
  uint64_t g = std::max<uint64_t>((bricks + per_wg - 1) / per_wg, std::min<uint64_t>(fine, 256));
  g = (g + 7) / 8 * 8;
  return static_cast<uint32_t>(std::min<uint64_t>(std::max<uint64_t>(g, 8), gbees::kMaxWG));
}

}  // namespace

struct gbees_ctx {
  gbees_config cfg;
  Layout L;
  char* base = nullptr;
  hipStream_t stream = nullptr;
  const KernelTable* kt = nullptr;
  Dev<double> d64;
  Dev<float> d32;
  const void* dev = nullptr;
  Scalars hsb;
  int status = GBEES_OK;
  uint32_t nb_est = 64;
  // Bricks per wave of the grid-stride launches: 8 for a grid that has the
  // device to itself; the serving pool uses 16, since its grids share the
  // device (measured on the serving stream: 8 per wave gave the best time for
  // requests run one at a time, 16 the best burst through the pool).
  uint32_t wave_bricks = 8;
  int64_t host_steps = 0;
  int batch = 4;
  gbees::Profiler prof;

  uint32_t G() const { return grid_for(std::max<uint32_t>(nb_est, 64), wave_bricks); }

  int sync_read() {
    if (hipMemcpyAsync(&hsb, base + L.sb, sizeof(Scalars), hipMemcpyDeviceToHost, stream) != hipSuccess)
      return fail(GBEES_E_DEVICE);
    if (hipStreamSynchronize(stream) != hipSuccess) return fail(GBEES_E_DEVICE);
    prof.harvest();
    return absorb();
  }
  // Host bookkeeping after a fresh copy of the scalar block landed in hsb.  A
  // grow that ran out of capacity or coordinate range is rolled back to the
  // start of its step: the error is returned and the context stays usable.
  int absorb() {
    nb_est = std::max<uint32_t>(std::min<uint32_t>(hsb.nb, L.cap_b), 64);
    host_steps = static_cast<int64_t>(hsb.steps);
    if (hsb.status == 0) return GBEES_OK;
    const int code = hsb.status == gbees::kErrRange ? GBEES_E_RANGE : GBEES_E_CAPACITY;
    if (hsb.status != gbees::kErrCapacity && hsb.status != gbees::kErrRange) return fail(code);
    kt->rollback(dev, stream, G());
    if (hipMemcpyAsync(&hsb, base + L.sb, sizeof(Scalars), hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
      return fail(GBEES_E_DEVICE);
    prof.harvest();
    nb_est = std::max<uint32_t>(std::min<uint32_t>(hsb.nb, L.cap_b), 64);
    host_steps = static_cast<int64_t>(hsb.steps);
    if (hsb.status != 0) return fail(code);
    return code;
  }
  // Enqueue up to K steps toward t_stop (steps past it are no-ops on the
  // device), with a prune or renormalisation after every prune_every-th step.
  void enqueue_steps(double t_stop, int K) {
    const bool prune_on = cfg.prune_every > 0;
    const bool thr_on = cfg.thresh_rel > 0.0;
    kt->set_tstop(dev, stream, t_stop);
    const uint32_t g = G();
    for (int k = 0; k < K; ++k) {
      kt->step(dev, stream, g, &prof);
      ++host_steps;
      if (prune_on && host_steps % cfg.prune_every == 0) {
        if (thr_on)
          kt->prune(dev, stream, g, true, &prof);
        else
          kt->normalise(dev, stream, g, gbees::kGateStep);
      }
    }
  }
  // Steps for the next batch: enough to reach t_stop at the last step size.
  void adapt_batch(double t_stop) {
    if (hsb.dt_last > 0.0) {
      const double est = std::ceil((t_stop - hsb.t) / hsb.dt_last);
      batch = static_cast<int>(std::min(std::max(est + 1.0, 1.0), 256.0));
    } else {
      batch = std::min(batch * 2, 256);
    }
  }
  int fail(int code) {
    if (status == GBEES_OK) status = code;
    return code;
  }
};

namespace {

// Copy the context's Dev block to its slot in the arena (read by launches that
// serve several grids).  Call again after every change to the host copy; the
// context must outlive the copy (it stays alive until its stream is synced).
bool upload_dev(gbees_ctx* c) {
  return hipMemcpyAsync(c->base + c->L.devc, c->dev, sizeof(gbees::Dev<double>), hipMemcpyHostToDevice, c->stream) ==
         hipSuccess;
}

// Delete a context whose stream may still hold work of new_ctx (clears and
// the upload of its Dev block, which reads the context itself).
void discard(gbees_ctx* c) {
  hipStreamSynchronize(c->stream);
  delete c;
}

gbees_ctx* new_ctx(const gbees_config* cfg, void* arena, size_t bytes, void* stream, int* err) {
  *err = GBEES_E_ARG;
  if (!cfg || !arena) return nullptr;
  Layout L;
  if (!make_layout(*cfg, &L) || bytes < L.total) return nullptr;
  auto* c = new (std::nothrow) gbees_ctx();
  if (!c) return nullptr;
  c->cfg = *cfg;
  c->L = L;
  c->base = static_cast<char*>(arena);
  c->stream = static_cast<hipStream_t>(stream);
  c->kt = gbees::kernel_table(effective_model(*cfg), cfg->n, cfg->precision);
  if (cfg->precision == 1) {
    fill_dev(c->d32, *cfg, L, c->base);
    c->dev = &c->d32;
  } else {
    fill_dev(c->d64, *cfg, L, c->base);
    c->dev = &c->d64;
  }
  std::memset(&c->hsb, 0, sizeof(c->hsb));
  if (hipMemsetAsync(c->base, 0, L.zero_end, c->stream) != hipSuccess ||
      hipMemsetAsync(c->base + L.zero_end, 0xFF, L.ff_end - L.zero_end, c->stream) != hipSuccess) {
    discard(c);
    *err = GBEES_E_DEVICE;
    return nullptr;
  }
  // The Dev block is uploaded by the caller once it is complete: the copy
  // reads the host block when it executes, so the block must not change
  // until the stream has passed it.
  *err = GBEES_OK;
  return c;
}

template <typename F>
void with_dev(gbees_ctx* c, F f) {
  if (c->cfg.precision == 1)
    f(c->d32);
  else
    f(c->d64);
}

int check_ctx(gbees_ctx* c) {
  if (!c) return GBEES_E_ARG;
  if (c->status != GBEES_OK) return GBEES_E_STATE;
  return GBEES_OK;
}

struct CellRow {
  int32_t idx[6];
  double p;
};

bool row_less(const CellRow& a, const CellRow& b, int n) {
  for (int j = 0; j < n; ++j)
    if (a.idx[j] != b.idx[j]) return a.idx[j] < b.idx[j];
  return false;
}

// Bricks of the current grid copied to the host and expanded to cells.
int host_cells(gbees_ctx* c, std::vector<CellRow>* rows) {
  const int rc = c->sync_read();
  if (rc != GBEES_OK) return rc;
  const uint32_t nb = std::min<uint32_t>(c->hsb.nb, c->L.cap_b);
  const int n = c->cfg.n;
  std::vector<u64> key(nb), mask(nb);
  std::vector<char> P(static_cast<size_t>(nb) * gbees::kLanes * c->L.real_size);
  const size_t poff = c->hsb.cur ? c->L.P1 : c->L.P0;
  if (nb > 0) {
    if (hipMemcpyAsync(key.data(), c->base + c->L.key, nb * 8, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipMemcpyAsync(mask.data(), c->base + c->L.mask, nb * 8, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipMemcpyAsync(P.data(), c->base + poff, P.size(), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
      return c->fail(GBEES_E_DEVICE);
  }
  rows->clear();
  for (uint32_t b = 0; b < nb; ++b) {
    int64_t B[6] = {0, 0, 0, 0, 0, 0};
    switch (n) {
      case 1: gbees::unpack_key<1>(key[b], B); break;
      case 2: gbees::unpack_key<2>(key[b], B); break;
      case 3: gbees::unpack_key<3>(key[b], B); break;
      case 4: gbees::unpack_key<4>(key[b], B); break;
      case 5: gbees::unpack_key<5>(key[b], B); break;
      default: gbees::unpack_key<6>(key[b], B); break;
    }
    for (int lane = 0; lane < gbees::kLanes; ++lane) {
      if (!((mask[b] >> lane) & 1ull)) continue;
      CellRow r;
      std::memset(&r, 0, sizeof(r));
      for (int j = 0; j < n; ++j) {
        const int a = (lane >> gbees::brick_off(n, j)) & (gbees::brick_side(n, j) - 1);
        r.idx[j] = static_cast<int32_t>(B[j] * gbees::brick_side(n, j) + a);
      }
      const size_t o = static_cast<size_t>(b) * gbees::kLanes + lane;
      r.p = c->L.real_size == 4 ? static_cast<double>(reinterpret_cast<const float*>(P.data())[o])
                                : reinterpret_cast<const double*>(P.data())[o];
      rows->push_back(r);
    }
  }
  std::sort(rows->begin(), rows->end(), [n](const CellRow& a, const CellRow& b) { return row_less(a, b, n); });
  return GBEES_OK;
}

template <int N>
u64 key_of_cell(const int32_t* idx, bool* ok) {
  int64_t B[N];
  for (int j = 0; j < N; ++j) {
    const int64_t i = idx[j];
    B[j] = (i >= 0) ? i / gbees::brick_side(N, j) : -((-i + gbees::brick_side(N, j) - 1) / gbees::brick_side(N, j));
  }
  *ok = gbees::brick_in_range<N>(B);
  return *ok ? gbees::pack_key<N>(B) : 0ull;
}

u64 key_of_cell_n(int n, const int32_t* idx, bool* ok) {
  switch (n) {
    case 1: return key_of_cell<1>(idx, ok);
    case 2: return key_of_cell<2>(idx, ok);
    case 3: return key_of_cell<3>(idx, ok);
    case 4: return key_of_cell<4>(idx, ok);
    case 5: return key_of_cell<5>(idx, ok);
    default: return key_of_cell<6>(idx, ok);
  }
}

// Validate, lay out the arena and enqueue the Gaussian initialisation (no wait).
int init_gaussian_begin(const gbees_config* cfg, void* arena, size_t arena_bytes, void* hip_stream, gbees_ctx** out) {
  if (!out) return GBEES_E_ARG;
  *out = nullptr;
  if (!cfg || !(cfg->thresh_rel > 0.0 && cfg->thresh_rel < 1.0)) return GBEES_E_ARG;
  double sinv[36];
  if (!spd_inverse(cfg->n, cfg->cov, sinv)) return GBEES_E_ARG;
  int err;
  gbees_ctx* c = new_ctx(cfg, arena, arena_bytes, hip_stream, &err);
  if (!c) return err;
  const int n = cfg->n;
  const double bound = 2.0 * std::log(1.0 / cfg->thresh_rel);
  int64_t lo[6] = {}, cnt[6] = {};
  double box = 1.0;
  for (int j = 0; j < n; ++j) {
    const int64_t r = static_cast<int64_t>(std::ceil(std::sqrt(bound * cfg->cov[j * n + j]) / cfg->h[j]));
    const int64_t side = gbees::brick_side(n, j);
    const int64_t blo = (-r >= 0) ? -r / side : -((r + side - 1) / side);
    const int64_t bhi = r / side;
    if (blo < -gbees::brick_limit(n) || bhi >= gbees::brick_limit(n)) {
      discard(c);
      return GBEES_E_RANGE;
    }
    lo[j] = blo;
    cnt[j] = bhi - blo + 1;
    box *= static_cast<double>(cnt[j]);
  }
  if (box > 4.0e12) {
    discard(c);
    return GBEES_E_ARG;
  }
  with_dev(c, [&](auto& d) {
    std::memcpy(d.sinv, sinv, sizeof(sinv));
    d.bound = bound;
    d.box_count = 1;
    for (int j = 0; j < n; ++j) {
      d.box_lo[j] = lo[j];
      d.box_n[j] = cnt[j];
      d.box_count *= static_cast<uint64_t>(cnt[j]);
    }
  });
  const uint64_t box_count = static_cast<uint64_t>(box);
  uint64_t gb = (box_count + 63) / 64;
  gb = std::min<uint64_t>(std::max<uint64_t>((gb + 7) / 8 * 8, 8), gbees::kMaxWG);
  c->nb_est = static_cast<uint32_t>(std::min<uint64_t>(box_count, c->L.cap_b));
  if (!upload_dev(c)) {
    discard(c);
    return GBEES_E_DEVICE;
  }
  c->kt->init_gaussian(c->dev, c->stream, c->G(), static_cast<uint32_t>(gb));
  *out = c;
  return GBEES_OK;
}


}  // namespace

extern "C" {

size_t gbees_arena_bytes(const gbees_config* cfg) {
  Layout L;
  if (!cfg || !make_layout(*cfg, &L)) return 0;
  return L.total;
}

int gbees_init_gaussian(const gbees_config* cfg, void* arena, size_t arena_bytes, void* hip_stream, gbees_ctx** out) {
  gbees_ctx* c = nullptr;
  int rc = init_gaussian_begin(cfg, arena, arena_bytes, hip_stream, &c);
  if (rc != GBEES_OK) return rc;
  rc = c->sync_read();
  if (rc != GBEES_OK) {
    discard(c);
    return rc;
  }
  *out = c;
  return GBEES_OK;
}

int gbees_init_cells(const gbees_config* cfg, const int32_t* idx, const double* P, int64_t count, double t0,
                     void* arena, size_t arena_bytes, void* hip_stream, gbees_ctx** out) {
  if (!out) return GBEES_E_ARG;
  *out = nullptr;
  if (!cfg || count < 0 || (count > 0 && (!idx || !P))) return GBEES_E_ARG;
  int err;
  gbees_ctx* c = new_ctx(cfg, arena, arena_bytes, hip_stream, &err);
  if (!c) return err;
  if (!upload_dev(c)) {
    discard(c);
    return GBEES_E_DEVICE;
  }
  const int n = cfg->n;
  // Group cells into bricks, bricks ordered by packed key.
  std::unordered_map<u64, uint32_t> where;
  std::vector<u64> keys;
  for (int64_t k = 0; k < count; ++k) {
    bool ok;
    const u64 key = key_of_cell_n(n, idx + k * n, &ok);
    if (!ok) {
      discard(c);
      return GBEES_E_RANGE;
    }
    if (where.emplace(key, 0u).second) keys.push_back(key);
  }
  std::sort(keys.begin(), keys.end());
  if (keys.size() > c->L.cap_b) {
    discard(c);
    return GBEES_E_CAPACITY;
  }
  for (size_t b = 0; b < keys.size(); ++b) where[keys[b]] = static_cast<uint32_t>(b);
  const size_t rs = c->L.real_size;
  std::vector<u64> mask(keys.size(), 0ull);
  std::vector<char> pbuf(keys.size() * gbees::kLanes * rs, 0);
  for (int64_t k = 0; k < count; ++k) {
    bool ok;
    const u64 key = key_of_cell_n(n, idx + k * n, &ok);
    const uint32_t b = where[key];
    int lane = 0;
    for (int j = 0; j < n; ++j) {
      const int32_t i = idx[k * n + j];
      const int side = gbees::brick_side(n, j);
      const int a = ((i % side) + side) % side;
      lane |= a << gbees::brick_off(n, j);
    }
    if ((mask[b] >> lane) & 1ull) {
      discard(c);
      return GBEES_E_ARG;  // duplicate cell
    }
    mask[b] |= 1ull << lane;
    const size_t o = static_cast<size_t>(b) * gbees::kLanes + lane;
    if (rs == 4)
      reinterpret_cast<float*>(pbuf.data())[o] = static_cast<float>(P[k]);
    else
      reinterpret_cast<double*>(pbuf.data())[o] = P[k];
  }
  Scalars s0;
  std::memset(&s0, 0, sizeof(s0));
  s0.nb = static_cast<uint32_t>(keys.size());
  s0.t = t0;
  s0.t_stop = t0;
  bool okc = true;
  if (!keys.empty()) {
    okc = hipMemcpyAsync(c->base + c->L.key, keys.data(), keys.size() * 8, hipMemcpyHostToDevice, c->stream) == hipSuccess &&
          hipMemcpyAsync(c->base + c->L.mask, mask.data(), mask.size() * 8, hipMemcpyHostToDevice, c->stream) == hipSuccess &&
          hipMemcpyAsync(c->base + c->L.abv, mask.data(), mask.size() * 8, hipMemcpyHostToDevice, c->stream) == hipSuccess &&
          hipMemcpyAsync(c->base + c->L.P0, pbuf.data(), pbuf.size(), hipMemcpyHostToDevice, c->stream) == hipSuccess;
  }
  okc = okc && hipMemcpyAsync(c->base + c->L.sb, &s0, sizeof(s0), hipMemcpyHostToDevice, c->stream) == hipSuccess;
  if (!okc) {
    discard(c);
    return GBEES_E_DEVICE;
  }
  c->nb_est = std::max<uint32_t>(s0.nb, 64);
  c->kt->init_finish(c->dev, c->stream, c->G());
  const int rc = c->sync_read();  // also keeps the host buffers alive until the copies finished
  if (rc != GBEES_OK) {
    discard(c);
    return rc;
  }
  *out = c;
  return GBEES_OK;
}

int gbees_step(gbees_ctx* c, double t_stop, int64_t max_steps, gbees_stats* out) {
  int rc = check_ctx(c);
  if (rc != GBEES_OK) return rc;
  if (!std::isfinite(t_stop) || t_stop < c->hsb.t) return GBEES_E_ARG;
  if (c->hsb.t < t_stop) {
    int64_t taken = 0;
    while (true) {
      int K = c->batch;
      if (max_steps > 0) K = static_cast<int>(std::min<int64_t>(K, max_steps - taken));
      const int64_t before = c->host_steps;
      c->enqueue_steps(t_stop, K);
      rc = c->sync_read();
      if (rc != GBEES_OK) return rc;
      taken += c->host_steps - before;
      if (c->hsb.t >= t_stop) break;
      if (max_steps > 0 && taken >= max_steps) break;
      c->adapt_batch(t_stop);
    }
  }
  return gbees_get_stats(c, out);
}

int gbees_correct(gbees_ctx* c, int32_t component, double y, double sigma) {
  const int rc = check_ctx(c);
  if (rc != GBEES_OK) return rc;
  if (component < 0 || component >= c->cfg.n || !(sigma > 0.0) || !std::isfinite(y)) return GBEES_E_ARG;
  const bool prune = c->cfg.prune_every > 0 && c->cfg.thresh_rel > 0.0;
  c->kt->correct(c->dev, c->stream, c->G(), component, y, sigma, prune);
  return c->sync_read();
}

int gbees_marginals(gbees_ctx* c, uint32_t dim_mask, int64_t capacity, int32_t* idx_out, double* val_out,
                    int64_t* count_out) {
  int rc = check_ctx(c);
  if (rc != GBEES_OK) return rc;
  const int n = c->cfg.n;
  if (dim_mask == 0 || (dim_mask >> n) != 0 || !count_out) return GBEES_E_ARG;
  rc = c->sync_read();
  if (rc != GBEES_OK) return rc;
  int nm = 0;
  for (int j = 0; j < n; ++j) nm += (dim_mask >> j) & 1u;
  const u64 cells = std::max<u64>(c->hsb.cells, 1);
  u64 tcap = 2;
  while (tcap < 2 * cells) tcap <<= 1;
  while (tcap > 2 && tcap * 32 > c->L.qbytes) tcap >>= 1;
  c->kt->marginals(c->dev, c->stream, c->G(), dim_mask, tcap - 1);
  rc = c->sync_read();
  if (rc != GBEES_OK) return rc;
  if (c->hsb.overflow) return GBEES_E_CAPACITY;
  const uint32_t count = c->hsb.nb_new;
  std::vector<u64> okey(count);
  std::vector<double> oval(count);
  const size_t off = c->L.Q + static_cast<size_t>(tcap) * 16;
  if (count > 0 &&
      (hipMemcpyAsync(okey.data(), c->base + off, count * 8, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
       hipMemcpyAsync(oval.data(), c->base + off + tcap * 8, count * 8, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
       hipStreamSynchronize(c->stream) != hipSuccess))
    return c->fail(GBEES_E_DEVICE);
  *count_out = count;
  if (capacity < static_cast<int64_t>(count)) return GBEES_E_BUFFER;
  if (count > 0 && (!idx_out || !val_out)) return GBEES_E_ARG;
  double w = 1.0;
  for (int j = 0; j < n; ++j)
    if (!((dim_mask >> j) & 1u)) w = w * c->cfg.h[j];
  const int kb = 63 / nm;
  const int64_t bias = int64_t(1) << (kb - 1);
  const u64 km = (kb >= 63) ? (~0ull >> 1) : ((1ull << kb) - 1);
  std::vector<CellRow> rows(count);
  for (uint32_t r = 0; r < count; ++r) {
    std::memset(&rows[r], 0, sizeof(CellRow));
    for (int q = 0; q < nm; ++q) rows[r].idx[q] = static_cast<int32_t>(static_cast<int64_t>((okey[r] >> (kb * q)) & km) - bias);
    rows[r].p = oval[r] * w;
  }
  std::sort(rows.begin(), rows.end(), [nm](const CellRow& a, const CellRow& b) { return row_less(a, b, nm); });
  for (uint32_t r = 0; r < count; ++r) {
    for (int q = 0; q < nm; ++q) idx_out[static_cast<size_t>(r) * nm + q] = rows[r].idx[q];
    val_out[r] = rows[r].p;
  }
  return GBEES_OK;
}

int gbees_marginals_noalloc(gbees_ctx* c, uint32_t dim_mask, int64_t capacity, int32_t* idx_dev, double* val_dev,
                            int64_t* count_dev) {
  const int rc = check_ctx(c);
  if (rc != GBEES_OK) return rc;
  const int n = c->cfg.n;
  if (dim_mask == 0 || (dim_mask >> n) != 0 || !count_dev || capacity < 0 || (capacity > 0 && (!idx_dev || !val_dev)))
    return GBEES_E_ARG;
  // The scalar block the host holds is current after every call that
  // returned; the table takes grids of up to half its slots in cells.
  if (c->hsb.cells > gbees::marginal_scratch_slots() / 2) return GBEES_E_CAPACITY;
  double w = 1.0;
  for (int j = 0; j < n; ++j)
    if (!((dim_mask >> j) & 1u)) w = w * c->cfg.h[j];
  if (!gbees::marginals_static(c->dev, n, c->cfg.precision, c->stream, c->G(), dim_mask, w, capacity, idx_dev, val_dev,
                               count_dev))
    return GBEES_E_DEVICE;
  return GBEES_OK;
}

int gbees_export(gbees_ctx* c, int64_t capacity, int32_t* idx, double* P, int64_t* count, double* t) {
  int rc = check_ctx(c);
  if (rc != GBEES_OK) return rc;
  if (!count) return GBEES_E_ARG;
  std::vector<CellRow> rows;
  rc = host_cells(c, &rows);
  if (rc != GBEES_OK) return rc;
  *count = static_cast<int64_t>(rows.size());
  if (t) *t = c->hsb.t;
  if (capacity < static_cast<int64_t>(rows.size())) return GBEES_E_BUFFER;
  if (!rows.empty() && (!idx || !P)) return GBEES_E_ARG;
  const int n = c->cfg.n;
  for (size_t r = 0; r < rows.size(); ++r) {
    for (int j = 0; j < n; ++j) idx[r * n + j] = rows[r].idx[j];
    P[r] = rows[r].p;
  }
  return GBEES_OK;
}

int gbees_get_stats(gbees_ctx* c, gbees_stats* out) {
  if (!c) return GBEES_E_ARG;
  if (c->status == GBEES_OK) {
    const int rc = c->sync_read();
    if (rc != GBEES_OK) return rc;
  } else {
    hipMemcpyAsync(&c->hsb, c->base + c->L.sb, sizeof(Scalars), hipMemcpyDeviceToHost, c->stream);
    hipStreamSynchronize(c->stream);
  }
  if (out) {
    double vol = 1.0;
    for (int j = 0; j < c->cfg.n; ++j) vol = vol * c->cfg.h[j];
    out->t = c->hsb.t;
    out->dt_last = c->hsb.dt_last;
    out->mass = vol * c->hsb.sum;
    out->max_p = c->hsb.maxp;
    double smax;
    std::memcpy(&smax, &c->hsb.smax_bits, sizeof(smax));
    out->smax = smax;
    out->steps = static_cast<int64_t>(c->hsb.steps);
    out->cell_updates = static_cast<int64_t>(c->hsb.cell_updates);
    out->brick_updates = static_cast<int64_t>(c->hsb.brick_updates);
    out->cells = static_cast<int64_t>(c->hsb.cells);
    out->bricks = static_cast<int64_t>(std::min<uint32_t>(c->hsb.nb, c->L.cap_b));
    out->prunes = static_cast<int64_t>(c->hsb.prunes);
    out->grow_bricks = static_cast<int64_t>(c->hsb.grow_bricks);
    out->inserted = static_cast<int64_t>(c->hsb.inserted);
    out->deferred = static_cast<int64_t>(c->hsb.deferred);
    out->mass_pruned = c->hsb.pruned;
  }
  return c->status;
}

int gbees_resize(gbees_ctx* c, int64_t max_cells, void* arena, size_t arena_bytes) {
  int rc = check_ctx(c);
  if (rc != GBEES_OK) return rc;
  if (!arena) return GBEES_E_ARG;
  gbees_config cfg = c->cfg;
  cfg.max_cells = max_cells;
  Layout L;
  if (!make_layout(cfg, &L) || arena_bytes < L.total) return GBEES_E_ARG;
  char* nb_base = static_cast<char*>(arena);
  if (nb_base < c->base + c->L.total && c->base < nb_base + L.total) return GBEES_E_ARG;  // overlap
  rc = c->sync_read();
  if (rc != GBEES_OK) return rc;
  const uint32_t nb = std::min<uint32_t>(c->hsb.nb, c->L.cap_b);
  if (nb > L.cap_b) return GBEES_E_CAPACITY;
  hipStream_t s = c->stream;
  const size_t rows = static_cast<size_t>(nb) * gbees::kLanes * c->L.real_size;
  Scalars sb = c->hsb;
  sb.cur = 0;
  bool ok = hipMemsetAsync(nb_base, 0, L.zero_end, s) == hipSuccess &&
            hipMemsetAsync(nb_base + L.zero_end, 0xFF, L.ff_end - L.zero_end, s) == hipSuccess;
  if (ok && nb > 0)
    ok = hipMemcpyAsync(nb_base + L.key, c->base + c->L.key, nb * 8, hipMemcpyDeviceToDevice, s) == hipSuccess &&
         hipMemcpyAsync(nb_base + L.mask, c->base + c->L.mask, nb * 8, hipMemcpyDeviceToDevice, s) == hipSuccess &&
         hipMemcpyAsync(nb_base + L.abv, c->base + c->L.mask, nb * 8, hipMemcpyDeviceToDevice, s) == hipSuccess &&
         hipMemcpyAsync(nb_base + L.done, c->base + c->L.done, nb * 8, hipMemcpyDeviceToDevice, s) == hipSuccess &&
         hipMemcpyAsync(nb_base + L.P0, c->base + (c->hsb.cur ? c->L.P1 : c->L.P0), rows, hipMemcpyDeviceToDevice,
                        s) == hipSuccess;
  ok = ok && hipMemcpyAsync(nb_base + L.sb, &sb, sizeof(sb), hipMemcpyHostToDevice, s) == hipSuccess;
  if (!ok) return c->fail(GBEES_E_DEVICE);
  // The context now describes the new arena; the initial-condition fields of
  // its Dev block carry over.
  with_dev(c, [&](auto& d) {
    auto keep = d;
    fill_dev(d, cfg, L, nb_base);
    std::memcpy(d.sinv, keep.sinv, sizeof(d.sinv));
    d.bound = keep.bound;
    std::memcpy(d.box_lo, keep.box_lo, sizeof(d.box_lo));
    std::memcpy(d.box_n, keep.box_n, sizeof(d.box_n));
    d.box_count = keep.box_count;
  });
  c->cfg = cfg;
  c->L = L;
  c->base = nb_base;
  if (!upload_dev(c)) return c->fail(GBEES_E_DEVICE);
  c->kt->relink(c->dev, s, c->G());
  return c->sync_read();  // also keeps sb alive until its copy finished
}

int gbees_probe_stats(gbees_ctx* c, int64_t n_miss, double* mean_hit, double* mean_miss, double* load) {
  int rc = check_ctx(c);
  if (rc != GBEES_OK) return rc;
  if (n_miss < 0) return GBEES_E_ARG;
  rc = c->sync_read();
  if (rc != GBEES_OK) return rc;
  double* out2 = reinterpret_cast<double*>(c->base + c->L.dpart);
  if (hipMemsetAsync(out2, 0, 2 * sizeof(double), c->stream) != hipSuccess) return c->fail(GBEES_E_DEVICE);
  c->kt->probe(c->dev, c->stream, c->G(), static_cast<uint64_t>(n_miss), out2);
  double h[2] = {0, 0};
  if (hipMemcpyAsync(h, out2, sizeof(h), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return c->fail(GBEES_E_DEVICE);
  const double nb = static_cast<double>(std::min<uint32_t>(c->hsb.nb, c->L.cap_b));
  if (mean_hit) *mean_hit = nb > 0 ? h[0] / nb : 0.0;
  if (mean_miss) *mean_miss = n_miss > 0 ? h[1] / static_cast<double>(n_miss) : 0.0;
  if (load) *load = nb / static_cast<double>(c->L.hcap);
  return GBEES_OK;
}

int gbees_profile(gbees_ctx* c, int enable) {
  if (!c) return GBEES_E_ARG;
  c->prof.on = enable != 0;
  return GBEES_OK;
}

int gbees_profile_read(gbees_ctx* c, double* ms, int64_t* launches) {
  if (!c) return GBEES_E_ARG;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return GBEES_E_DEVICE;
  c->prof.harvest();
  for (int k = 0; k < gbees::kProfKinds; ++k) {
    if (ms) ms[k] = c->prof.ms[k];
    if (launches) launches[k] = c->prof.launches[k];
    c->prof.ms[k] = 0.0;
    c->prof.launches[k] = 0;
  }
  return GBEES_OK;
}

int gbees_destroy(gbees_ctx* c) {
  if (!c) return GBEES_E_ARG;
  hipStreamSynchronize(c->stream);
  c->prof.release();
  delete c;
  return GBEES_OK;
}

const char* gbees_strerror(int code) {
  switch (code) {
    case GBEES_OK: return "ok";
    case GBEES_E_ARG: return "invalid argument";
    case GBEES_E_CAPACITY: return "grid capacity exceeded";
    case GBEES_E_RANGE: return "cell index out of the packable range";
    case GBEES_E_DEVICE: return "HIP runtime error";
    case GBEES_E_BUFFER: return "output buffer too small";
    case GBEES_E_STATE: return "context is in an error state";
    default: return "unknown error";
  }
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Serving pool: many propagation requests share one caller-owned arena.
// Each admitted request gets a slice of the arena sized by its footprint
// (gbees_arena_bytes of its configuration) and runs through the same steps as
// the single-grid calls: initialise, step to each measurement time, correct,
// step to the horizon.  Running requests of one kind are stepped together by
// their group's driver thread with shared launches (PoolGroup); requests of
// different kinds overlap on the device through their groups' streams.
// gbees_pool_progress admits waiting requests in arrival order as slots and
// arena slices become free; it never waits on the device.
// ---------------------------------------------------------------------------
namespace {

using PoolClock = std::chrono::steady_clock;

// First-fit allocator over [0, bytes) of the pool arena (host bookkeeping only).
class SliceAllocator {
 public:
  explicit SliceAllocator(size_t bytes) { free_.push_back({0, bytes}); }
  bool take(size_t bytes, size_t* off) {
    bytes = align_up(bytes);
    for (size_t k = 0; k < free_.size(); ++k) {
      if (free_[k].size >= bytes) {
        *off = free_[k].off;
        free_[k].off += bytes;
        free_[k].size -= bytes;
        if (free_[k].size == 0) free_.erase(free_.begin() + static_cast<std::ptrdiff_t>(k));
        return true;
      }
    }
    return false;
  }
  void give(size_t off, size_t bytes) {
    bytes = align_up(bytes);
    auto it = std::lower_bound(free_.begin(), free_.end(), off, [](const Span& s, size_t o) { return s.off < o; });
    it = free_.insert(it, Span{off, bytes});
    if (it + 1 != free_.end() && it->off + it->size == (it + 1)->off) {
      it->size += (it + 1)->size;
      free_.erase(it + 1);
    }
    if (it != free_.begin() && (it - 1)->off + (it - 1)->size == it->off) {
      (it - 1)->size += it->size;
      free_.erase(it);
    }
  }

 private:
  struct Span {
    size_t off, size;
  };
  std::vector<Span> free_;
};

struct PoolRequest {
  gbees_config cfg{};
  double t_end = 0.0;
  std::vector<gbees_meas> meas;  // sorted by time, within [0, t_end]
  size_t bytes = 0, off = 0;
  int32_t status = 0;  // 0 waiting, 1 running, 2 done, < 0 error code
  hipStream_t stream = nullptr;
  gbees_ctx* ctx = nullptr;
  double t_submit = 0.0, t_admit = 0.0, t_done = 0.0;
  gbees_stats stats{};
  std::vector<CellRow> rows;
  bool exporting = false;  // a gbees_pool_result call is copying the grid out
  bool exported = false;
  int64_t resizes = 0;     // moves into a larger arena slice after the grid outgrew its capacity
};

// A request's place in its group's run: the context, the next measurement
// and the time it is stepping to.
struct Runner {
  int64_t id;
  PoolRequest* r;
  gbees_ctx* c;
  size_t k;  // next measurement (k == meas.size(): stepping to t_end)
  double target() const { return k < r->meas.size() ? r->meas[k].t : r->t_end; }
};

}  // namespace

// Requests of one kind (model, dimension, precision) advance together: a
// driver thread steps the running requests of its group with shared launches
// (KernelTable::step_multi), so K steps of R grids cost 7K launches instead of
// 7KR.  Each grid keeps its own workgroup count and device state, so it
// computes what it would compute alone with that workgroup count; only the
// number of steps per batch (the smallest any member asks for) is shared, and
// steps past a grid's stop time are no-ops on the device.  A pooled grid's
// launches use 16 bricks per wave (8 alone): the same cells and densities up to
// the rounding of its sums, which are partitioned over other workgroups.
constexpr uint32_t kPoolWaveBricks = 16;  // bricks per wave of a pooled grid's launches

struct PoolGroup {
  int model = 0, n = 0, precision = 0;
  int members = 0;  // admitted and not finished (guarded by the pool mutex)
  const gbees::KernelTable* kt = nullptr;
  hipStream_t stream = nullptr;
  std::deque<int64_t> inbox;  // admitted, not yet initialised (guarded by the pool mutex)
  std::thread th;
};

struct gbees_pool {
  // Requests per driver: enough to share launches, few enough that several
  // drivers of one kind overlap on the device while one of them waits for its
  // batch, reads back scalars or corrects.  (gbees_pool_group_size sets it.)
  int per_driver = 4;
  char* base = nullptr;
  size_t total = 0;
  SliceAllocator slices{0};
  std::mutex mu;
  std::condition_variable work_cv;
  std::condition_variable export_cv;  // a result copy finished
  std::deque<int64_t> pending;  // waiting for a slot and a slice
  std::unordered_map<int64_t, PoolRequest> reqs;
  std::vector<std::unique_ptr<PoolGroup>> groups;
  int busy = 0, max_active = 0;
  bool stop = false;
  int64_t next_id = 1;
  int device = 0;
  PoolClock::time_point t0 = PoolClock::now();

  double now() const { return std::chrono::duration<double>(PoolClock::now() - t0).count(); }

  // The group of the request's kind with the fewest members, or a new one if
  // each has per_driver.  (Caller holds mu.)
  PoolGroup* group_for(const gbees_config& cfg) {
    const int model = effective_model(cfg), prec = cfg.precision == 1 ? 1 : 0;
    PoolGroup* best = nullptr;
    for (auto& g : groups)
      if (g->model == model && g->n == cfg.n && g->precision == prec && g->members < per_driver &&
          (!best || g->members < best->members))
        best = g.get();
    if (best) return best;
    auto g = std::make_unique<PoolGroup>();
    g->model = model;
    g->n = cfg.n;
    g->precision = prec;
    g->kt = gbees::kernel_table(model, cfg.n, prec);
    if (!g->kt || hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking) != hipSuccess) return nullptr;
    PoolGroup* raw = g.get();
    groups.push_back(std::move(g));
    raw->th = std::thread([this, raw] { drive(*raw); });
    return raw;
  }

  // Scalar blocks of every context in cs, with one wait on the group stream.
  static int read_all(PoolGroup& g, const std::vector<gbees_ctx*>& cs) {
    for (gbees_ctx* c : cs)
      if (hipMemcpyAsync(&c->hsb, c->base + c->L.sb, sizeof(Scalars), hipMemcpyDeviceToHost, g.stream) != hipSuccess)
        return GBEES_E_DEVICE;
    if (hipStreamSynchronize(g.stream) != hipSuccess) return GBEES_E_DEVICE;
    return GBEES_OK;
  }

  // A runner left its group (done or failed): its context moves to the
  // request's own stream for the export and release.  Every exit comes right
  // after a wait on the group stream (the batch read-back, a correction or the
  // final statistics), so no group work for this grid is still pending.
  void leave(PoolGroup& g, Runner& x, int rc) {
    if (rc != GBEES_OK) (void)hipStreamSynchronize(g.stream);  // an error may have cut a wait short
    if (x.c) x.c->stream = x.r->stream;
    std::lock_guard<std::mutex> lk(mu);
    x.r->t_done = now();
    x.r->status = rc == GBEES_OK ? 2 : rc;
    if (rc != GBEES_OK) free_request(*x.r);
    --busy;
    --g.members;
  }

  // A runner whose grid outgrew its capacity (its last step was rolled back):
  // move it into a slice four, else two, times as large and keep it running.
  // False if no slice that large is free now.
  bool enlarge(Runner& x) {
    PoolRequest& r = *x.r;
    for (int64_t factor : {4, 2}) {
      gbees_config cfg = r.cfg;
      cfg.max_cells = r.cfg.max_cells * factor;
      const size_t bytes = gbees_arena_bytes(&cfg);
      if (bytes == 0) continue;
      size_t off = 0;
      {
        std::lock_guard<std::mutex> lk(mu);
        if (!slices.take(bytes, &off)) continue;
      }
      const int rc = gbees_resize(x.c, cfg.max_cells, base + off, bytes);
      std::lock_guard<std::mutex> lk(mu);
      if (rc != GBEES_OK) {
        slices.give(off, bytes);
        return false;
      }
      slices.give(r.off, r.bytes);
      r.off = off;
      r.bytes = bytes;
      r.cfg.max_cells = cfg.max_cells;
      ++r.resizes;
      return true;
    }
    return false;
  }

  // Measurements due now (t reached), then the end: corrections and exits.
  // Returns false when the runner is finished (left the group).
  bool advance(PoolGroup& g, Runner& x) {
    while (x.c->hsb.t >= x.target()) {
      if (x.k == x.r->meas.size()) {
        const int rc = gbees_get_stats(x.c, &x.r->stats);
        leave(g, x, rc);
        return false;
      }
      const gbees_meas& m = x.r->meas[x.k];
      const int rc = gbees_correct(x.c, m.component, m.y, m.sigma);
      if (rc != GBEES_OK) {
        leave(g, x, rc);
        return false;
      }
      ++x.k;
    }
    return true;
  }

  void drive(PoolGroup& g) {
    hipSetDevice(device);
    std::vector<Runner> run;
    while (true) {
      std::vector<int64_t> fresh;
      {
        std::unique_lock<std::mutex> lk(mu);
        work_cv.wait(lk, [&] { return stop || !g.inbox.empty() || !run.empty(); });
        if (stop && g.inbox.empty() && run.empty()) return;
        fresh.assign(g.inbox.begin(), g.inbox.end());
        g.inbox.clear();
      }
      // Initialise the newcomers on the group stream.
      std::vector<Runner> born;
      for (int64_t id : fresh) {
        PoolRequest* r;
        {
          std::lock_guard<std::mutex> lk(mu);
          r = &reqs[id];
        }
        Runner x{id, r, nullptr, 0};
        const int rc = init_gaussian_begin(&r->cfg, base + r->off, r->bytes, g.stream, &x.c);
        if (x.c) x.c->wave_bricks = kPoolWaveBricks;
        r->ctx = x.c;
        if (rc != GBEES_OK) {
          leave(g, x, rc);
          continue;
        }
        born.push_back(x);
      }
      if (!born.empty()) {
        std::vector<gbees_ctx*> cs;
        for (auto& x : born) cs.push_back(x.c);
        const int rc = read_all(g, cs);
        for (auto& x : born) {
          const int rx = rc != GBEES_OK ? rc : x.c->absorb();
          if (rx != GBEES_OK)
            leave(g, x, rx);
          else if (advance(g, x))
            run.push_back(x);
        }
      }
      if (run.empty()) continue;
      // One batch of K shared steps toward each runner's own target.
      int K = 256;
      for (auto& x : run) {
        K = std::min(K, x.c->batch);
        x.c->kt->set_tstop(x.c->dev, g.stream, x.target());
      }
      for (size_t at = 0; at < run.size(); at += gbees::kMultiMax) {
        const size_t R = std::min<size_t>(gbees::kMultiMax, run.size() - at);
        gbees::MultiGrids m{};
        m.R = static_cast<uint32_t>(R);
        m.wg0[0] = 0;
        for (size_t i = 0; i < R; ++i) {
          gbees_ctx* c = run[at + i].c;
          m.dev[i] = c->base + c->L.devc;
          m.wg0[i + 1] = m.wg0[i] + c->G();
        }
        for (int k = 0; k < K; ++k) {
          g.kt->step_multi(m, g.stream);
          for (size_t i = 0; i < R; ++i) {
            gbees_ctx* c = run[at + i].c;
            if (c->cfg.prune_every > 0 && ++c->host_steps % c->cfg.prune_every == 0)
              c->kt->prune(c->dev, g.stream, c->G(), true, &c->prof);
          }
        }
      }
      std::vector<gbees_ctx*> cs;
      for (auto& x : run) cs.push_back(x.c);
      const int rc = read_all(g, cs);
      std::vector<Runner> keep;
      for (auto& x : run) {
        const int rx = rc != GBEES_OK ? rc : x.c->absorb();
        if (rx == GBEES_E_CAPACITY && x.c->status == GBEES_OK && enlarge(x)) {
          keep.push_back(x);
          continue;
        }
        if (rx != GBEES_OK) {
          leave(g, x, rx);
          continue;
        }
        if (!advance(g, x)) continue;
        x.c->adapt_batch(x.target());
        keep.push_back(x);
      }
      run.swap(keep);
    }
  }

  // Give back the device side of a request (caller holds mu or owns r).
  void free_request(PoolRequest& r) {
    if (r.ctx) {
      gbees_destroy(r.ctx);
      r.ctx = nullptr;
    }
    if (r.stream) {
      hipStreamDestroy(r.stream);
      r.stream = nullptr;
      slices.give(r.off, r.bytes);
    }
  }
};

extern "C" {

int gbees_pool_create(void* arena, size_t arena_bytes, int32_t max_active, gbees_pool** out) {
  if (!out || !arena || arena_bytes < kAlign || max_active < 1 || max_active > 256) return GBEES_E_ARG;
  *out = nullptr;
  auto* p = new (std::nothrow) gbees_pool();
  if (!p) return GBEES_E_ARG;
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return GBEES_E_DEVICE;
  }
  p->base = static_cast<char*>(arena);
  p->total = arena_bytes / kAlign * kAlign;
  p->slices = SliceAllocator(p->total);
  p->max_active = max_active;
  *out = p;
  return GBEES_OK;
}

int gbees_pool_submit(gbees_pool* p, const gbees_config* cfg, double t_end, const gbees_meas* meas, int32_t nm,
                      int64_t* req) {
  if (!p || !cfg || !req || nm < 0 || (nm > 0 && !meas) || !std::isfinite(t_end) || t_end < 0.0) return GBEES_E_ARG;
  const size_t bytes = gbees_arena_bytes(cfg);
  if (bytes == 0 || !(cfg->thresh_rel > 0.0) || cfg->grow_mode == 2) return GBEES_E_ARG;
  if (align_up(bytes) > p->total) return GBEES_E_CAPACITY;  // could never be admitted
  PoolRequest r;
  r.cfg = *cfg;
  r.t_end = t_end;
  for (int32_t k = 0; k < nm; ++k) {
    const gbees_meas& m = meas[k];
    if (m.component < 0 || m.component >= cfg->n || !(m.sigma > 0.0) || !std::isfinite(m.y) || !(m.t >= 0.0))
      return GBEES_E_ARG;
    if (m.t <= t_end) r.meas.push_back(m);
  }
  std::stable_sort(r.meas.begin(), r.meas.end(), [](const gbees_meas& a, const gbees_meas& b) { return a.t < b.t; });
  r.bytes = bytes;
  std::lock_guard<std::mutex> lk(p->mu);
  r.t_submit = p->now();
  const int64_t id = p->next_id++;
  p->reqs.emplace(id, std::move(r));
  p->pending.push_back(id);
  *req = id;
  return GBEES_OK;
}

int gbees_pool_progress(gbees_pool* p, int32_t* n_running, int32_t* n_waiting) {
  if (!p) return GBEES_E_ARG;
  int admitted = 0;
  int rc = GBEES_OK;
  {
    std::lock_guard<std::mutex> lk(p->mu);
    // Admit in arrival order; a request that does not fit may be passed by the
    // next three.
    for (auto it = p->pending.begin(); it != p->pending.end() && p->busy < p->max_active;) {
      PoolRequest& r = p->reqs[*it];
      size_t off = 0;
      if (!p->slices.take(r.bytes, &off)) {
        if (it - p->pending.begin() >= 3) break;
        ++it;
        continue;
      }
      PoolGroup* g = p->group_for(r.cfg);
      if (!g || hipStreamCreateWithFlags(&r.stream, hipStreamNonBlocking) != hipSuccess) {
        p->slices.give(off, r.bytes);
        r.stream = nullptr;
        rc = GBEES_E_DEVICE;
        break;
      }
      r.off = off;
      r.status = 1;
      r.t_admit = p->now();
      g->inbox.push_back(*it);
      ++g->members;
      ++p->busy;
      ++admitted;
      it = p->pending.erase(it);
    }
    if (n_running) *n_running = p->busy;
    if (n_waiting) *n_waiting = static_cast<int32_t>(p->pending.size());
  }
  if (admitted) p->work_cv.notify_all();
  return rc;
}

int gbees_pool_info(gbees_pool* p, int64_t req, gbees_req_info* out) {
  if (!p || !out) return GBEES_E_ARG;
  std::lock_guard<std::mutex> lk(p->mu);
  auto it = p->reqs.find(req);
  if (it == p->reqs.end()) return GBEES_E_ARG;
  const PoolRequest& r = it->second;
  out->status = r.status;
  out->t_submit = r.t_submit;
  out->t_admit = r.t_admit;
  out->t_done = r.t_done;
  out->arena_bytes = static_cast<int64_t>(r.bytes);
  out->cells = r.status == 2 ? r.stats.cells : 0;
  std::memset(&out->stats, 0, sizeof(out->stats));
  if (r.status == 2) out->stats = r.stats;
  out->resizes = r.resizes;
  return GBEES_OK;
}

int gbees_pool_result(gbees_pool* p, int64_t req, int64_t capacity, int32_t* idx, double* P, int64_t* count) {
  if (!p || !count) return GBEES_E_ARG;
  std::unique_lock<std::mutex> lk(p->mu);
  auto it = p->reqs.find(req);
  if (it == p->reqs.end()) return GBEES_E_ARG;
  PoolRequest& r = it->second;
  if (r.status < 0) return r.status;
  if (r.status != 2) return GBEES_E_STATE;
  // A concurrent call for the same request waits for the first one's copy.
  p->export_cv.wait(lk, [&] { return !r.exporting; });
  if (!r.exported) {
    // First call: copy the grid out (outside the lock: the drivers keep running)
    // and free the device side.  The exporting flag keeps every other call
    // (result or release) off the context meanwhile.
    gbees_ctx* c = r.ctx;
    r.exporting = true;
    lk.unlock();
    std::vector<CellRow> rows;
    const int rc = host_cells(c, &rows);
    lk.lock();
    r.exporting = false;
    p->export_cv.notify_all();
    if (rc != GBEES_OK) return rc;
    r.rows = std::move(rows);
    r.exported = true;
    p->free_request(r);
  }
  *count = static_cast<int64_t>(r.rows.size());
  if (capacity < *count) return GBEES_E_BUFFER;
  if (*count > 0 && (!idx || !P)) return GBEES_E_ARG;
  const int n = r.cfg.n;
  for (size_t k = 0; k < r.rows.size(); ++k) {
    for (int j = 0; j < n; ++j) idx[k * n + j] = r.rows[k].idx[j];
    P[k] = r.rows[k].p;
  }
  return GBEES_OK;
}

int gbees_pool_release(gbees_pool* p, int64_t req) {
  if (!p) return GBEES_E_ARG;
  std::lock_guard<std::mutex> lk(p->mu);
  auto it = p->reqs.find(req);
  if (it == p->reqs.end()) return GBEES_E_ARG;
  PoolRequest& r = it->second;
  if (r.status == 0 || r.status == 1 || r.exporting) return GBEES_E_STATE;
  p->free_request(r);
  p->reqs.erase(it);
  return GBEES_OK;
}

int gbees_pool_group_size(gbees_pool* p, int32_t k) {
  if (!p || k < 1 || k > gbees::kMultiMax) return GBEES_E_ARG;
  std::lock_guard<std::mutex> lk(p->mu);
  p->per_driver = k;
  return GBEES_OK;
}

double gbees_pool_clock(gbees_pool* p) { return p ? p->now() : 0.0; }

int gbees_pool_destroy(gbees_pool* p) {
  if (!p) return GBEES_E_ARG;
  {
    std::lock_guard<std::mutex> lk(p->mu);
    p->stop = true;
    p->pending.clear();  // never admitted
  }
  p->work_cv.notify_all();
  for (auto& g : p->groups) g->th.join();  // running requests finish first
  for (auto& kv : p->reqs) p->free_request(kv.second);
  for (auto& g : p->groups) hipStreamDestroy(g->stream);
  delete p;
  return GBEES_OK;
}

}  // extern "C"
