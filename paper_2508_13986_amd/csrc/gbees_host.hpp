// Host-side internals shared by the kernel launchers and the C ABI.
#pragma once

#include <vector>

#include "gbees_dev.hpp"

namespace gbees {

enum ProfKind { kProfGrow = 0, kProfGrowFix, kProfFluxA, kProfFluxB, kProfPrune, kProfOther, kProfKinds };

// Optional per-pass device timing with HIP events on the launch stream.
struct Profiler {
  bool on = false;
  std::vector<hipEvent_t> ev;   // pairs: 2k start, 2k+1 stop
  std::vector<int> kind;
  size_t used = 0;
  double ms[kProfKinds] = {};
  long long launches[kProfKinds] = {};

  void begin(int k, hipStream_t s) {
    if (!on) return;
    if (2 * used + 2 > ev.size()) {
      for (int i = 0; i < 64; ++i) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return;
        ev.push_back(e);
      }
      kind.resize(ev.size() / 2);
    }
    kind[used] = k;
    hipEventRecord(ev[2 * used], s);
  }
  void end(hipStream_t s) {
    if (!on || 2 * used + 2 > ev.size()) return;
    hipEventRecord(ev[2 * used + 1], s);
    ++used;
  }
  // Call after the stream has been synchronised.
  void harvest() {
    for (size_t i = 0; i < used; ++i) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, ev[2 * i], ev[2 * i + 1]) == hipSuccess) {
        ms[kind[i]] += t;
        launches[kind[i]] += 1;
      }
    }
    used = 0;
  }
  void release() {
    for (hipEvent_t e : ev) hipEventDestroy(e);
    ev.clear();
    kind.clear();
    used = 0;
  }
};

// Launch sequences of one (model, dimension, precision) instantiation.  `dev`
// points to a Dev<double> or Dev<float> matching the precision.
// Grids of one kind stepped by shared launches: grid r owns workgroups
// [wg0[r], wg0[r + 1]) of every grid-wide launch (a multiple of 8 each, the
// count it would be launched with alone) and dev[r] is the device copy of its
// Dev block.  Passed by value as the kernels' argument.
constexpr int kMultiMax = 64;
struct MultiGrids {
  const void* dev[kMultiMax];
  uint32_t wg0[kMultiMax + 1];
  uint32_t R;
};

struct KernelTable {
  int n, model, precision;
  // Full initial grid from the ellipsoid box, then hashtable, links, speed, normalisation.
  void (*init_gaussian)(const void* dev, hipStream_t s, uint32_t G, uint32_t G_box);
  // After bricks were copied in: hashtable, links, speed, max (no normalisation).
  void (*init_finish)(const void* dev, hipStream_t s, uint32_t G);
  // One time step (gated on the device by t < t_stop and status == ok).
  void (*step)(const void* dev, hipStream_t s, uint32_t G, Profiler* pf);
  // Prune + compaction + rehash + relink + normalisation.  from_step: run only
  // if the preceding step ran.
  void (*prune)(const void* dev, hipStream_t s, uint32_t G, bool from_step, Profiler* pf);
  void (*correct)(const void* dev, hipStream_t s, uint32_t G, int comp, double y, double sigma, bool prune);
  void (*normalise)(const void* dev, hipStream_t s, uint32_t G, int gate);
  void (*set_tstop)(const void* dev, hipStream_t s, double t_stop);
  // Marginal: projected-key aggregation into a scratch table, compacted to [0, count).
  void (*marginals)(const void* dev, hipStream_t s, uint32_t G, uint32_t dim_mask, uint64_t table_mask);
  void (*probe)(const void* dev, hipStream_t s, uint32_t G, uint64_t n_miss, double* out2);
  // One time step of every grid in m (each gated on its own device state), as
  // `step` would take it alone with its own workgroup count.
  void (*step_multi)(const MultiGrids& m, hipStream_t s);
  // After a grow that failed for lack of capacity or coordinate range: the
  // grid as it was when that step began, with a clear status.
  void (*rollback)(const void* dev, hipStream_t s, uint32_t G);
  // Hashtable and axis links rebuilt from the brick keys and masks.
  void (*relink)(const void* dev, hipStream_t s, uint32_t G);
};

const KernelTable* kernel_table(int model, int n, int precision);

// Marginals through the file-scope scratch table of noalloc.hip (no
// allocation, no host copy, no wait): slots of that table, and the launcher.
uint64_t marginal_scratch_slots();
bool marginals_static(const void* dev, int n, int precision, hipStream_t s, uint32_t G, uint32_t dim_mask,
                      double weight, int64_t capacity, int32_t* idx, double* val, int64_t* count);

}  // namespace gbees
