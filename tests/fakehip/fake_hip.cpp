// A host-only stand-in for the HIP runtime and the kernel launch table, used
// to run the library's host code (gbees.cpp: contexts, step batching, the
// serving pool and its driver threads) on the CPU under AddressSanitizer and
// ThreadSanitizer.  TEST INFRASTRUCTURE ONLY; nothing of the method is here.
//
// Streams are worker threads that run their queue in order, so copies and
// "kernels" happen after the call that enqueued them returns, as on a GPU:
// a copy reads and writes host memory when it executes, and a kernel takes its
// Dev block by value at launch (like kernel arguments) and works on the arena,
// which is ordinary host memory here.  The fake kernels keep the scalar block
// consistent (time, steps, brick counts, status) with a toy grid that gains a
// brick every third step, so capacity errors, rollbacks, resizes, exports and
// corrections take the same host paths as on the device.
#include <hip/hip_runtime.h>

#include <atomic>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <functional>
#include <mutex>
#include <thread>

#include "gbees_host.hpp"

namespace {

struct FakeStream {
  std::mutex mu;
  std::condition_variable cv, idle_cv;
  std::deque<std::function<void()>> q;
  bool busy = false, stop = false;
  std::thread th;

  FakeStream() : th([this] { run(); }) {}
  ~FakeStream() {
    {
      std::lock_guard<std::mutex> lk(mu);
      stop = true;
    }
    cv.notify_all();
    th.join();
  }
  void run() {
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
      cv.wait(lk, [&] { return stop || !q.empty(); });
      if (q.empty() && stop) return;
      auto f = std::move(q.front());
      q.pop_front();
      busy = true;
      lk.unlock();
      f();
      lk.lock();
      busy = false;
      if (q.empty()) idle_cv.notify_all();
    }
  }
  void push(std::function<void()> f) {
    {
      std::lock_guard<std::mutex> lk(mu);
      q.push_back(std::move(f));
    }
    cv.notify_one();
  }
  void drain() {
    std::unique_lock<std::mutex> lk(mu);
    idle_cv.wait(lk, [&] { return q.empty() && !busy; });
  }
};

FakeStream& null_stream() {
  static FakeStream s;
  return s;
}
FakeStream& S(hipStream_t s) { return s ? *reinterpret_cast<FakeStream*>(s) : null_stream(); }

thread_local int g_device = 0;

}  // namespace

extern "C" {

hipError_t hipSetDevice(int d) {
  g_device = d;
  return hipSuccess;
}
hipError_t hipGetDevice(int* d) {
  *d = g_device;
  return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned int) {
  *s = reinterpret_cast<hipStream_t>(new FakeStream());
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  if (!s) return hipErrorInvalidValue;
  FakeStream* f = reinterpret_cast<FakeStream*>(s);
  f->drain();
  delete f;
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
  S(s).drain();
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind, hipStream_t s) {
  S(s).push([=] { std::memcpy(dst, src, n); });
  return hipSuccess;
}
hipError_t hipMemsetAsync(void* dst, int v, size_t n, hipStream_t s) {
  S(s).push([=] { std::memset(dst, v, n); });
  return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
  *ms = 0.f;
  return hipSuccess;
}

}  // extern "C"

namespace gbees {
namespace {

template <typename Real>
struct Fake {
  static Dev<Real> D(const void* p) { return *static_cast<const Dev<Real>*>(p); }
  static double bits(u64 b) {
    double v;
    std::memcpy(&v, &b, 8);
    return v;
  }
  static u64 to_bits(double v) {
    u64 b;
    std::memcpy(&b, &v, 8);
    return b;
  }
  static Real* cur(const Dev<Real>& d) { return d.sb->cur ? d.P1 : d.P0; }

  // A brick of 64 cells at index b: key b, every lane present, density p.
  static void put_brick(const Dev<Real>& d, uint32_t b, Real p) {
    d.key[b] = b;
    d.mask[b] = ~0ull;
    for (int l = 0; l < kLanes; ++l) cur(d)[static_cast<size_t>(b) * kLanes + l] = p;
  }
  static void totals(const Dev<Real>& d) {
    Scalars* sb = d.sb;
    const uint32_t nb = sb->nb < d.cap_b ? sb->nb : d.cap_b;
    double s = 0.0, m = 0.0;
    for (size_t i = 0; i < static_cast<size_t>(nb) * kLanes; ++i) {
      s += static_cast<double>(cur(d)[i]);
      m = static_cast<double>(cur(d)[i]) > m ? static_cast<double>(cur(d)[i]) : m;
    }
    sb->sum = s;
    sb->maxp = m;
    sb->cells = static_cast<u64>(nb) * kLanes;
  }
  static void step_one(const Dev<Real>& d) {
    Scalars* sb = d.sb;
    sb->run = (sb->status == 0 && sb->t < sb->t_stop) ? 1u : 0u;
    if (sb->status == 0) {
      sb->nb_old = sb->nb;
      sb->smax_begin = sb->smax_bits;
    }
    if (!sb->run) return;
    if ((sb->steps + 1) % 3 == 0) {  // grow one brick
      const uint32_t b = sb->nb++;
      if (b >= d.cap_b) {
        sb->status = kErrCapacity;
        sb->run = 0;
        return;
      }
      put_brick(d, b, Real(0));
    }
    const double rem = sb->t_stop - sb->t, dt = 0.0125;
    sb->dt = dt >= rem ? rem : dt;
    sb->t = dt >= rem ? sb->t_stop : sb->t + dt;
    sb->dt_last = sb->dt;
    sb->steps += 1;
    sb->cell_updates += static_cast<u64>(sb->nb) * kLanes;
    sb->brick_updates += sb->nb;
    totals(d);
  }

  static void init_gaussian(const void* p, hipStream_t s, uint32_t, uint32_t) {
    const Dev<Real> d = D(p);
    S(s).push([d] {
      const uint32_t nb = 2 + static_cast<uint32_t>(d.box_count % 5);
      d.sb->nb = nb;
      if (nb > d.cap_b) {
        d.sb->status = kErrCapacity;
        return;
      }
      for (uint32_t b = 0; b < nb; ++b) put_brick(d, b, static_cast<Real>(1.0 / (d.vol * kLanes * nb)));
      for (uint32_t b = 0; b < nb; ++b) d.abv[b] = d.mask[b];
      d.sb->smax_bits = to_bits(1.0);
      totals(d);
    });
  }
  static void init_finish(const void* p, hipStream_t s, uint32_t) {
    const Dev<Real> d = D(p);
    S(s).push([d] { totals(d); });
  }
  static void step(const void* p, hipStream_t s, uint32_t, Profiler*) {
    const Dev<Real> d = D(p);
    S(s).push([d] { step_one(d); });
  }
  static void prune(const void* p, hipStream_t s, uint32_t, bool from_step, Profiler*) {
    const Dev<Real> d = D(p);
    S(s).push([d, from_step] {
      Scalars* sb = d.sb;
      sb->prun = (sb->status == 0 && (!from_step || sb->run)) ? 1u : 0u;
      if (sb->prun) sb->prunes += 1;
    });
  }
  static void correct(const void* p, hipStream_t s, uint32_t G, int, double, double, bool do_prune) {
    const Dev<Real> d = D(p);
    S(s).push([d] { totals(d); });
    if (do_prune) prune(p, s, G, false, nullptr);
  }
  static void normalise(const void* p, hipStream_t s, uint32_t, int) {
    const Dev<Real> d = D(p);
    S(s).push([d] { totals(d); });
  }
  static void set_tstop(const void* p, hipStream_t s, double t) {
    const Dev<Real> d = D(p);
    S(s).push([d, t] { d.sb->t_stop = t; });
  }
  static void marginals(const void* p, hipStream_t s, uint32_t, uint32_t, uint64_t tmask) {
    const Dev<Real> d = D(p);
    S(s).push([d, tmask] {
      d.sb->nb_new = 1;
      d.sb->overflow = 0;
      u64* okey = reinterpret_cast<u64*>(reinterpret_cast<char*>(d.Q) + (tmask + 1) * 16);
      okey[0] = 0;
      reinterpret_cast<double*>(okey + tmask + 1)[0] = 1.0;
    });
  }
  static void probe(const void*, hipStream_t s, uint32_t, uint64_t, double* out2) {
    S(s).push([out2] { out2[0] = out2[1] = 1.0; });
  }
  static void step_multi(const MultiGrids& m, hipStream_t s) {
    const MultiGrids mm = m;
    // Each grid's Dev block is read from its device copy when the "kernel" runs.
    S(s).push([mm] {
      for (uint32_t r = 0; r < mm.R; ++r) step_one(*static_cast<const Dev<Real>*>(mm.dev[r]));
    });
  }
  static void rollback(const void* p, hipStream_t s, uint32_t) {
    const Dev<Real> d = D(p);
    S(s).push([d] {
      Scalars* sb = d.sb;
      if (sb->status != kErrCapacity && sb->status != kErrRange) return;
      for (uint32_t b = sb->nb_old; b < sb->nb && b < d.cap_b; ++b) d.mask[b] = 0;
      sb->nb = sb->nb_old;
      sb->smax_bits = sb->smax_begin;
      sb->status = 0;
      sb->run = sb->prun = 0;
      totals(d);
    });
  }
  static void relink(const void* p, hipStream_t s, uint32_t) {
    const Dev<Real> d = D(p);
    S(s).push([d] { totals(d); });
  }
  static KernelTable entry(int n, int model, int prec) {
    return {n,          model,      prec,   &init_gaussian, &init_finish, &step,     &prune,   &correct,
            &normalise, &set_tstop, &marginals, &probe,     &step_multi,  &rollback, &relink};
  }
};

struct Tables {
  KernelTable t[2][4][7];
  Tables() {
    for (int m = 1; m <= 3; ++m)
      for (int n = 1; n <= 6; ++n) {
        t[0][m][n] = Fake<double>::entry(n, m, 0);
        t[1][m][n] = Fake<float>::entry(n, m, 1);
      }
  }
};

}  // namespace

uint64_t marginal_scratch_slots() { return uint64_t(1) << 20; }
bool marginals_static(const void*, int, int, hipStream_t, uint32_t, uint32_t, double, int64_t, int32_t*, double*,
                      int64_t*) {
  return false;
}

const KernelTable* kernel_table(int model, int n, int precision) {
  static const Tables tables;
  if (precision != 0 && precision != 1) return nullptr;
  if (model < 1 || model > 3 || n < 1 || n > 6) return nullptr;
  return &tables.t[precision][model][n];
}

}  // namespace gbees
