// GBEES time-step oracle: a plain, slow, single-threaded FP64 CPU implementation.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or calls
// this file; only the test-suite, the smoke check and the CPU-baseline leg of the
// benchmark use it.  It shares no source, header, table or helper with the HIP path.
//
// What it computes (GBEES-GPU, arXiv 2508.13986):
//   * the sparse grid is a std::unordered_map from the integer multi-index i of a
//     control volume (Sec. 2.1, Eq. 5) to its cell-average density P_i;
//   * one time step is: threshold -> directional grow -> CFL time step -> Donor
//     Cell Upwind fluxes (Eq. 7) -> Corner Transport Upwind corrections applied
//     literally in scatter form (Algorithm 1) -> optional high-resolution term ->
//     conservative update -> optional directional prune + renormalisation
//     (Sec. 3.2-3.3, Eq. 8, Algorithm 3);
//   * a Bayesian measurement correction (Eq. 4) with a scalar Gaussian likelihood;
//   * lower-dimensional marginals by summing out coordinates (Sec. 5.1.2).
//
// Readings taken where the paper is silent (each also listed in the design notes):
//   R1 a face contributes to the update only when both of its cells are in the grid;
//   R2 dt = C / max_i sum_j |f_{i-1/2 e_j, j}| / h_j over the grown grid, clamped so
//      that t lands exactly on the stop time;
//   R3 high-resolution term: one-dimensional MC-limited correction per face
//      (LeVeque, Finite Volume Methods for Hyperbolic Problems, ch. 6), no
//      transverse propagation of it; limiter 0 gives exactly Eq. 7 + Algorithm 1;
//   R4 grow/prune neighbour set: axis neighbours plus pairwise edge neighbours,
//      chosen by the sign of the face velocity (downwind for grow, upwind for prune);
//      grow_mode 2 takes every combination of those steps (the orthant, Sec. 3.3);
//   R5 grow uses set semantics over the pre-grow grid; new cells do not grow;
//   R6 p* = thresh_rel * max P; P == p* counts as above; zero velocity is neither
//      up- nor downwind; with thresh_rel = 0 every non-zero cell grows (never prunes);
//   R8 P is a cell-average density, normalised so that V * sum P = 1, V = prod h_j;
//   R9 cell centres are x_i = mean + i*h; the initial grid is every lattice point of
//      the ellipsoid q(i) <= 2 ln(1/thresh_rel), P = exp(-q/2), normalised;
//   R11 face-centre coordinates are mean_j + (i_j - 1/2) h_j; the drift is evaluated
//      in a fixed operation order with floating-point contraction disabled.
//
// Build: g++ -O2 -std=c++17 -ffp-contract=off -shared -fPIC (see oracle/build.py).

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <unordered_map>
#include <vector>

namespace {

constexpr int kMaxDim = 6;

enum Model { kL63 = 1, kL96 = 2, kLinear = 3, kUniform = 4 };

struct Idx {
  std::array<int32_t, kMaxDim> c{};
  bool operator==(const Idx& o) const { return c == o.c; }
};

struct IdxHash {
  size_t operator()(const Idx& k) const {
    uint64_t h = 1469598103934665603ull;
    for (int d = 0; d < kMaxDim; ++d) {
      h ^= static_cast<uint32_t>(k.c[d]);
      h *= 1099511628211ull;
    }
    return static_cast<size_t>(h);
  }
};

using Grid = std::unordered_map<Idx, double, IdxHash>;

}  // namespace

extern "C" {

// Mirrors the fields the Python wrapper fills in; independent of any product header.
struct oracle_config {
  int32_t n;             // dimension, 1..6
  int32_t model;         // 1 Lorenz-63, 2 Lorenz-96, 3 linear f = A x + b, 4 uniform f = b
  double params[48];     // L63: sigma, rho, beta, z_shift; L96: F; linear: A (n*n row-major), b (n); uniform: b (n)
  double h[6];           // cell widths
  double mean[6];        // initial mean; also the grid anchor (centre of cell 0)
  double cov[36];        // initial covariance, row-major n*n, symmetric positive definite
  double thresh_rel;     // p* = thresh_rel * max P; 0 => grow from P != 0, never prune
  double cfl;            // Courant number C
  double dt_fixed;       // > 0 overrides the CFL step
  int32_t prune_every;   // prune after every prune_every-th step; 0 = never
  int32_t limiter;       // 0 none (Eq. 7 + Algorithm 1 only), 1 MC-limited high-resolution term
  int32_t grow_mode;     // 0 directional (R4), 1 every axis and pairwise-edge neighbour,
                         // 2 directional over the whole orthant (every combination of downwind steps)
};

struct oracle_stats {
  double t;
  double dt_last;
  double min_margin;     // min |P - p*| / max P over every threshold decision so far
  double mass;           // V * sum P
  int64_t steps;
  int64_t cell_updates;  // sum over steps of the number of cells updated
  int64_t cells;         // current number of cells
  int64_t prunes;
};

}  // extern "C"

namespace {

struct StepLog {
  double t, dt, smax, maxp, min_margin;
  int64_t cells;
};

struct Oracle {
  oracle_config cfg;
  Grid grid;
  double t = 0.0;
  double dt_last = 0.0;
  double min_margin = std::numeric_limits<double>::infinity();
  double step_margin = std::numeric_limits<double>::infinity();
  int64_t steps = 0;
  int64_t cell_updates = 0;
  int64_t prunes = 0;
  std::vector<StepLog> log;

  int n() const { return cfg.n; }

  // ---- geometry (Eq. 5, R9, R11) ----
  double centre(int j, int32_t i) const { return cfg.mean[j] + static_cast<double>(i) * cfg.h[j]; }
  double face_coord(int j, int32_t i) const { return cfg.mean[j] + (static_cast<double>(i) - 0.5) * cfg.h[j]; }

  // ---- drift f(x) (Sec. 5.1.1, 5.1.2; the linear and uniform fields are test drifts) ----
  double drift(const double* x, int j) const {
    const double* p = cfg.params;
    const int nn = cfg.n;
    switch (cfg.model) {
      case kL63: {
        // Lorenz '63 standard form evaluated at (x1, x2, x3 + z_shift); with
        // rho = r and z_shift = r it is the shifted form printed in Sec. 5.1.1.
        const double z = x[2] + p[3];
        if (j == 0) return p[0] * (x[1] - x[0]);
        if (j == 1) return x[0] * (p[1] - z) - x[1];
        return x[0] * x[1] - p[2] * z;
      }
      case kL96: {
        // Lorenz '96, cyclic indices (Sec. 5.1.2).
        const int jp1 = (j + 1) % nn, jm1 = (j + nn - 1) % nn, jm2 = (j + nn - 2) % nn;
        return (x[jp1] - x[jm2]) * x[jm1] - x[j] + p[0];
      }
      case kLinear: {
        double acc = p[j * nn + 0] * x[0];
        for (int k = 1; k < nn; ++k) acc = acc + p[j * nn + k] * x[k];
        return acc + p[nn * nn + j];
      }
      case kUniform:
        return p[j];
      default:
        return 0.0;
    }
  }

  // f_j at the centre of the backward j-face of cell i: f_{i - 1/2 e_j, j}.
  double face_vel(const Idx& i, int j) const {
    double x[kMaxDim] = {0, 0, 0, 0, 0, 0};
    for (int m = 0; m < n(); ++m) x[m] = (m == j) ? face_coord(m, i.c[m]) : centre(m, i.c[m]);
    return drift(x, j);
  }

  static Idx shift(const Idx& i, int j, int s) {
    Idx o = i;
    o.c[j] += s;
    return o;
  }
  static Idx shift2(const Idx& i, int j, int s, int l, int r) {
    Idx o = i;
    o.c[j] += s;
    o.c[l] += r;
    return o;
  }

  double P(const Idx& i) const {
    auto it = grid.find(i);
    return it == grid.end() ? 0.0 : it->second;
  }
  bool has(const Idx& i) const { return grid.count(i) != 0; }

  double max_p() const {
    double m = 0.0;
    for (const auto& kv : grid) m = std::max(m, kv.second);
    return m;
  }

  double volume() const {
    double v = 1.0;
    for (int j = 0; j < n(); ++j) v = v * cfg.h[j];
    return v;
  }

  void note_margin(double p, double pstar, double m) {
    if (cfg.thresh_rel <= 0.0 || m <= 0.0) return;
    const double g = std::fabs(p - pstar) / m;
    step_margin = std::min(step_margin, g);
    min_margin = std::min(min_margin, g);
  }

  // Sum of every density, compensated (Neumaier's improvement of Kahan
  // summation): a running sum over N cells can be off by about N * 1.1e-16
  // relative, which at 1e7 cells exceeds the 1e-12 to which densities are
  // compared; the compensated sum is accurate to a few units in the last place.
  double sum_p() const {
    double s = 0.0, c = 0.0;
    for (const auto& kv : grid) {
      const double v = kv.second, t = s + v;
      c += (std::fabs(s) >= std::fabs(v)) ? (s - t) + v : (v - t) + s;
      s = t;
    }
    return s + c;
  }

  // R8: scale so that V * sum P = 1.
  void normalise() {
    const double z = volume() * sum_p();
    if (z > 0.0)
      for (auto& kv : grid) kv.second = kv.second / z;
  }

  // ---- initial condition (R9) ----
  int init_gaussian() {
    const int nn = n();
    if (cfg.thresh_rel <= 0.0 || cfg.thresh_rel >= 1.0) return -1;
    // Inverse covariance by Gauss-Jordan elimination with partial pivoting.
    double a[kMaxDim][2 * kMaxDim];
    for (int r = 0; r < nn; ++r)
      for (int c = 0; c < 2 * nn; ++c) a[r][c] = (c < nn) ? cfg.cov[r * nn + c] : (c - nn == r ? 1.0 : 0.0);
    for (int col = 0; col < nn; ++col) {
      int piv = col;
      for (int r = col + 1; r < nn; ++r)
        if (std::fabs(a[r][col]) > std::fabs(a[piv][col])) piv = r;
      if (a[piv][col] == 0.0) return -1;
      if (piv != col)
        for (int c = 0; c < 2 * nn; ++c) std::swap(a[piv][c], a[col][c]);
      const double d = a[col][col];
      for (int c = 0; c < 2 * nn; ++c) a[col][c] = a[col][c] / d;
      for (int r = 0; r < nn; ++r) {
        if (r == col) continue;
        const double f = a[r][col];
        if (f == 0.0) continue;
        for (int c = 0; c < 2 * nn; ++c) a[r][c] = a[r][c] - f * a[col][c];
      }
    }
    double sinv[kMaxDim][kMaxDim];
    for (int r = 0; r < nn; ++r)
      for (int c = 0; c < nn; ++c) sinv[r][c] = a[r][c + nn];

    const double bound = 2.0 * std::log(1.0 / cfg.thresh_rel);
    int32_t rad[kMaxDim] = {0, 0, 0, 0, 0, 0};
    for (int j = 0; j < nn; ++j)
      rad[j] = static_cast<int32_t>(std::ceil(std::sqrt(bound * cfg.cov[j * nn + j]) / cfg.h[j]));

    grid.clear();
    Idx i;
    for (int j = 0; j < nn; ++j) i.c[j] = -rad[j];
    while (true) {
      double y[kMaxDim];
      for (int j = 0; j < nn; ++j) y[j] = static_cast<double>(i.c[j]) * cfg.h[j];
      double q = 0.0;
      for (int j = 0; j < nn; ++j) {
        double row = 0.0;
        for (int k = 0; k < nn; ++k) row = row + sinv[j][k] * y[k];
        q = q + y[j] * row;
      }
      if (q <= bound) grid[i] = std::exp(-q / 2.0);
      int d = 0;
      while (d < nn) {
        if (i.c[d] < rad[d]) {
          ++i.c[d];
          break;
        }
        i.c[d] = -rad[d];
        ++d;
      }
      if (d == nn) break;
    }
    normalise();
    t = 0.0;
    return 0;
  }

  // Orthant neighbour set (grow_mode 2, Sec. 3.3 and Figs. 2-3: every
  // neighbour on the downwind side, up to 2^n - 1 of them): c plus any
  // non-zero combination of steps, at most one per dimension, each step
  // +e_j allowed when plus[j] and -e_j when minus[j].
  void orthant(const Idx& c, const bool* plus, const bool* minus, std::vector<Idx>& out) const {
    const int nn = n();
    int step[kMaxDim] = {0, 0, 0, 0, 0, 0};
    // Odometer over the per-dimension choices {0, +1, -1} that are allowed.
    while (true) {
      int j = 0;
      while (j < nn) {
        const int next = step[j] == 0 ? +1 : (step[j] == +1 ? -1 : 2);
        if (next == +1 && plus[j]) { step[j] = +1; break; }
        if ((next == +1 || next == -1) && minus[j]) { step[j] = -1; break; }
        step[j] = 0;
        ++j;
      }
      if (j == nn) return;
      Idx o = c;
      for (int m = 0; m < nn; ++m) o.c[m] += step[m];
      out.push_back(o);
    }
  }

  // ---- directional grow (Sec. 3.3, R4, R5, R6) ----
  void grow_candidates(const Idx& c, std::vector<Idx>& out) const {
    const int nn = n();
    bool up[kMaxDim], dn[kMaxDim];  // downwind sets: +1 if f at forward face > 0, -1 if f at backward face < 0
    for (int j = 0; j < nn; ++j) {
      if (cfg.grow_mode == 1) {
        up[j] = dn[j] = true;
      } else {
        up[j] = face_vel(shift(c, j, +1), j) > 0.0;
        dn[j] = face_vel(c, j) < 0.0;
      }
    }
    if (cfg.grow_mode == 2) {
      orthant(c, up, dn, out);
      return;
    }
    for (int j = 0; j < nn; ++j) {
      if (up[j]) out.push_back(shift(c, j, +1));
      if (dn[j]) out.push_back(shift(c, j, -1));
    }
    for (int j = 0; j < nn; ++j)
      for (int l = j + 1; l < nn; ++l)
        for (int s = -1; s <= 1; s += 2)
          for (int r = -1; r <= 1; r += 2) {
            const bool sj = (s > 0) ? up[j] : dn[j];
            const bool rl = (r > 0) ? up[l] : dn[l];
            if (sj && rl) out.push_back(shift2(c, j, s, l, r));
          }
  }

  // With thresh_rel = 0 every cell holding any (non-zero) density is a grow source.
  bool above(double p, double pstar) const { return cfg.thresh_rel > 0.0 ? p >= pstar : p != 0.0; }

  int64_t grow() {
    const double m = max_p();
    const double pstar = cfg.thresh_rel * m;
    std::vector<Idx> cand;
    for (const auto& kv : grid) {
      note_margin(kv.second, pstar, m);
      if (above(kv.second, pstar)) grow_candidates(kv.first, cand);
    }
    int64_t added = 0;
    for (const Idx& c : cand)
      if (grid.emplace(c, 0.0).second) ++added;
    return added;
  }

  // ---- CFL time step (Eq. 8, R2) ----
  double smax() const {
    double s_max = 0.0;
    for (const auto& kv : grid) {
      double s = 0.0;
      for (int j = 0; j < n(); ++j) s = s + std::fabs(face_vel(kv.first, j)) / cfg.h[j];
      s_max = std::max(s_max, s);
    }
    return s_max;
  }

  // ---- fluxes: Eq. 7, then Algorithm 1 literally, then R3 ----
  static double pos(double v) { return v > 0.0 ? v : 0.0; }
  static double neg(double v) { return v < 0.0 ? v : 0.0; }

  static double mc_limited(double w, double wup) {
    if (w * wup <= 0.0) return 0.0;
    const double m = std::min(std::fabs(w + wup) / 2.0, std::min(2.0 * std::fabs(w), 2.0 * std::fabs(wup)));
    return w > 0.0 ? m : -m;
  }

  // Face fluxes of one step.  Only a face whose two cells are both in the grid
  // enters the update (R1), and such a face is the backward face of a grid
  // cell, so the fluxes are kept per grid cell: F[i][j] is the flux through the
  // face between i - e_j and i.  Contributions to faces of cells outside the
  // grid are dropped.
  using FluxMap = std::unordered_map<Idx, std::array<double, kMaxDim>, IdxHash>;

  static void add_flux(FluxMap& F, const Idx& c, int j, double v) {
    auto it = F.find(c);
    if (it != F.end()) it->second[j] += v;
  }

  void fluxes(double dt, FluxMap& F) const {
    const int nn = n();
    // Donor Cell Upwind (Eq. 7): the flux through each backward face carries
    // the density of the cell the face velocity comes from.
    for (const auto& kv : grid) {
      const Idx& i = kv.first;
      std::array<double, kMaxDim> f{};
      for (int j = 0; j < nn; ++j) {
        const double u = face_vel(i, j);
        f[j] = pos(u) * P(shift(i, j, -1)) + neg(u) * kv.second;
      }
      F.emplace(i, f);
    }
    // Corner Transport Upwind (Algorithm 1).  The jump of P across the
    // backward j-face of cell i is a wave moving with the face velocity a.  It
    // enters the cell on the downwind side of that face (i when a > 0, i - e_j
    // when a < 0).  Inside that cell, half the wave times dt / h_j is carried
    // on along each other direction l by the velocity at the cell's l-faces:
    // out through the forward l-face where that velocity is positive, out
    // through the backward l-face where it is negative.  The face flux changes
    // by -a * v * dt / (2 h_j) * jump, v being the velocity at that face.
    for (const auto& kv : grid) {
      const Idx& i = kv.first;
      for (int j = 0; j < nn; ++j) {
        const double a = face_vel(i, j);
        if (a == 0.0) continue;
        const Idx into = (a > 0.0) ? i : shift(i, j, -1);
        const double w = dt / (2.0 * cfg.h[j]) * (kv.second - P(shift(i, j, -1)));
        for (int l = 0; l < nn; ++l) {
          if (l == j) continue;
          const Idx ahead = shift(into, l, +1);
          const double v_fwd = face_vel(ahead, l);  // velocity at the forward l-face of `into`
          const double v_bwd = face_vel(into, l);   // velocity at its backward l-face
          if (v_fwd > 0.0) add_flux(F, ahead, l, -(a * v_fwd * w));
          if (v_bwd < 0.0) add_flux(F, into, l, -(a * v_bwd * w));
        }
      }
    }
    // High-resolution correction (R3): limited second-order term per face.
    if (cfg.limiter == 1) {
      for (const auto& kv : grid) {
        const Idx& i = kv.first;
        for (int j = 0; j < nn; ++j) {
          const double u = face_vel(i, j);
          if (u == 0.0) continue;
          const double w = kv.second - P(shift(i, j, -1));
          const double wup = (u > 0.0) ? P(shift(i, j, -1)) - P(shift(i, j, -2)) : P(shift(i, j, +1)) - kv.second;
          const double au = std::fabs(u);
          F.at(i)[j] += 0.5 * au * (1.0 - dt * au / cfg.h[j]) * mc_limited(w, wup);
        }
      }
    }
  }

  // ---- one time step ----
  int step_once(double t_stop) {
    step_margin = std::numeric_limits<double>::infinity();
    grow();
    const double s_max = smax();
    const double rem = t_stop - t;
    double dt;
    if (cfg.dt_fixed > 0.0)
      dt = cfg.dt_fixed;
    else
      dt = (s_max > 0.0) ? cfg.cfl / s_max : rem;
    const bool last = dt >= rem;
    if (last) dt = rem;

    FluxMap F;
    F.reserve(grid.size());
    fluxes(dt, F);

    Grid next;
    next.reserve(grid.size());
    for (const auto& kv : grid) {
      const Idx& i = kv.first;
      double acc = kv.second;
      const auto& own = F.at(i);
      for (int j = 0; j < n(); ++j) {
        const double dth = dt / cfg.h[j];
        if (has(shift(i, j, -1))) acc += dth * own[j];
        const auto ahead = F.find(shift(i, j, +1));
        if (ahead != F.end()) acc -= dth * ahead->second[j];
      }
      next.emplace(i, acc);
    }
    cell_updates += static_cast<int64_t>(grid.size());
    grid.swap(next);

    t = last ? t_stop : t + dt;
    dt_last = dt;
    ++steps;
    const int64_t cells_updated = static_cast<int64_t>(grid.size());
    if (cfg.prune_every > 0 && steps % cfg.prune_every == 0) prune();
    log.push_back(StepLog{t, dt, s_max, max_p(), step_margin, cells_updated});
    return 0;
  }

  // ---- directional prune (Sec. 3.3, Algorithm 3, R4, R6) + renormalisation ----
  void prune() {
    if (cfg.thresh_rel <= 0.0) {
      normalise();
      return;
    }
    const double m = max_p();
    const double pstar = cfg.thresh_rel * m;
    const int nn = n();
    std::vector<Idx> dead;
    for (const auto& kv : grid) {
      const Idx& i = kv.first;
      note_margin(kv.second, pstar, m);
      if (kv.second >= pstar) continue;
      bool up[kMaxDim], dn[kMaxDim];  // upwind sets: +1 if f at forward face < 0, -1 if f at backward face > 0
      for (int j = 0; j < nn; ++j) {
        up[j] = face_vel(shift(i, j, +1), j) < 0.0;
        dn[j] = face_vel(i, j) > 0.0;
      }
      bool keep = false;
      auto check = [&](const Idx& u) {
        auto it = grid.find(u);
        if (it == grid.end()) return;
        note_margin(it->second, pstar, m);
        if (it->second >= pstar) keep = true;
      };
      if (cfg.grow_mode == 2) {
        std::vector<Idx> ups;
        orthant(i, up, dn, ups);
        for (const Idx& u : ups) check(u);
        if (!keep) dead.push_back(i);
        continue;
      }
      for (int j = 0; j < nn; ++j) {
        if (up[j]) check(shift(i, j, +1));
        if (dn[j]) check(shift(i, j, -1));
      }
      for (int j = 0; j < nn; ++j)
        for (int l = j + 1; l < nn; ++l)
          for (int s = -1; s <= 1; s += 2)
            for (int r = -1; r <= 1; r += 2) {
              const bool sj = (s > 0) ? up[j] : dn[j];
              const bool rl = (r > 0) ? up[l] : dn[l];
              if (sj && rl) check(shift2(i, j, s, l, r));
            }
      if (!keep) dead.push_back(i);
    }
    for (const Idx& d : dead) grid.erase(d);
    normalise();
    ++prunes;
  }

  // ---- Bayesian correction (Eq. 4) with y = x_c + noise, noise ~ N(0, sigma^2) ----
  int correct(int comp, double y, double sigma) {
    if (comp < 0 || comp >= n() || !(sigma > 0.0)) return -1;
    for (auto& kv : grid) {
      const double d = y - centre(comp, kv.first.c[comp]);
      const double e = (d * d) / (2.0 * sigma * sigma);
      kv.second = kv.second * std::exp(-e);
    }
    if (cfg.prune_every > 0 && cfg.thresh_rel > 0.0)
      prune();
    else
      normalise();
    return 0;
  }

  std::vector<Idx> sorted_keys() const {
    std::vector<Idx> keys;
    keys.reserve(grid.size());
    for (const auto& kv : grid) keys.push_back(kv.first);
    std::sort(keys.begin(), keys.end(), [](const Idx& a, const Idx& b) { return a.c < b.c; });
    return keys;
  }
};

}  // namespace

extern "C" {

void* oracle_new(const oracle_config* cfg) {
  if (!cfg || cfg->n < 1 || cfg->n > kMaxDim) return nullptr;
  auto* o = new Oracle();
  o->cfg = *cfg;
  return o;
}

void oracle_free(void* h) { delete static_cast<Oracle*>(h); }

int oracle_init_gaussian(void* h) { return static_cast<Oracle*>(h)->init_gaussian(); }

// Cells given by the caller (row-major count x n indices and their densities).
int oracle_init_cells(void* h, const int32_t* idx, const double* p, int64_t count, double t0) {
  auto* o = static_cast<Oracle*>(h);
  o->grid.clear();
  for (int64_t k = 0; k < count; ++k) {
    Idx i;
    for (int j = 0; j < o->n(); ++j) i.c[j] = idx[k * o->n() + j];
    o->grid[i] = p[k];
  }
  o->t = t0;
  return 0;
}

// Advance until t == t_stop (or max_steps internal steps, when max_steps > 0).
int oracle_step(void* h, double t_stop, int64_t max_steps) {
  auto* o = static_cast<Oracle*>(h);
  int64_t k = 0;
  while (o->t < t_stop && (max_steps <= 0 || k < max_steps)) {
    o->step_once(t_stop);
    ++k;
  }
  return 0;
}

// The grow phase alone (for set tests); returns the number of cells added.
int64_t oracle_grow(void* h) { return static_cast<Oracle*>(h)->grow(); }

// The prune phase alone (including its renormalisation).
void oracle_prune(void* h) { static_cast<Oracle*>(h)->prune(); }

void oracle_normalise(void* h) { static_cast<Oracle*>(h)->normalise(); }

double oracle_smax(void* h) { return static_cast<Oracle*>(h)->smax(); }

int oracle_correct(void* h, int32_t comp, double y, double sigma) {
  return static_cast<Oracle*>(h)->correct(comp, y, sigma);
}

int64_t oracle_count(void* h) { return static_cast<int64_t>(static_cast<Oracle*>(h)->grid.size()); }

// Cells sorted lexicographically by index; returns the count written or -needed.
int64_t oracle_export(void* h, int32_t* idx, double* p, int64_t cap) {
  auto* o = static_cast<Oracle*>(h);
  const auto keys = o->sorted_keys();
  const int64_t cnt = static_cast<int64_t>(keys.size());
  if (cnt > cap) return -cnt;
  for (int64_t k = 0; k < cnt; ++k) {
    for (int j = 0; j < o->n(); ++j) idx[k * o->n() + j] = keys[k].c[j];
    p[k] = o->grid.at(keys[k]);
  }
  return cnt;
}

// Marginal over the dimensions in dim_mask: M(k) = sum_{i: i_mask = k} P_i * prod_{j not in mask} h_j.
int64_t oracle_marginals(void* h, uint32_t dim_mask, int32_t* idx, double* val, int64_t cap) {
  auto* o = static_cast<Oracle*>(h);
  const int nn = o->n();
  double w = 1.0;
  for (int j = 0; j < nn; ++j)
    if (!(dim_mask >> j & 1u)) w = w * o->cfg.h[j];
  Grid acc;
  for (const auto& kv : o->grid) {
    Idx k;
    for (int j = 0; j < nn; ++j) k.c[j] = (dim_mask >> j & 1u) ? kv.first.c[j] : 0;
    acc[k] += kv.second;
  }
  std::vector<Idx> keys;
  for (const auto& kv : acc) keys.push_back(kv.first);
  std::sort(keys.begin(), keys.end(), [](const Idx& a, const Idx& b) { return a.c < b.c; });
  const int64_t cnt = static_cast<int64_t>(keys.size());
  if (cnt > cap) return -cnt;
  int m = 0;
  for (int j = 0; j < nn; ++j) m += (dim_mask >> j & 1u) ? 1 : 0;
  for (int64_t r = 0; r < cnt; ++r) {
    int c = 0;
    for (int j = 0; j < nn; ++j)
      if (dim_mask >> j & 1u) idx[r * m + c++] = keys[r].c[j];
    val[r] = acc.at(keys[r]) * w;
  }
  return cnt;
}

void oracle_get_stats(void* h, oracle_stats* s) {
  auto* o = static_cast<Oracle*>(h);
  const double sum = o->sum_p();
  s->t = o->t;
  s->dt_last = o->dt_last;
  s->min_margin = o->min_margin;
  s->mass = o->volume() * sum;
  s->steps = o->steps;
  s->cell_updates = o->cell_updates;
  s->cells = static_cast<int64_t>(o->grid.size());
  s->prunes = o->prunes;
}

// Per-step log rows: t, dt, smax, max P, step margin, cells updated (6 doubles each).
int64_t oracle_log(void* h, double* out, int64_t cap_rows) {
  auto* o = static_cast<Oracle*>(h);
  const int64_t rows = static_cast<int64_t>(o->log.size());
  if (rows > cap_rows) return -rows;
  for (int64_t r = 0; r < rows; ++r) {
    const StepLog& L = o->log[r];
    out[r * 6 + 0] = L.t;
    out[r * 6 + 1] = L.dt;
    out[r * 6 + 2] = L.smax;
    out[r * 6 + 3] = L.maxp;
    out[r * 6 + 4] = L.min_margin;
    out[r * 6 + 5] = static_cast<double>(L.cells);
  }
  return rows;
}

// Drift f_j at an arbitrary point (model pins).
double oracle_drift(void* h, const double* x, int32_t j) { return static_cast<Oracle*>(h)->drift(x, j); }

// Face velocity f_{i - 1/2 e_j, j} for a cell index (pins of the face-coordinate convention).
double oracle_face_vel(void* h, const int32_t* idx, int32_t j) {
  auto* o = static_cast<Oracle*>(h);
  Idx i;
  for (int d = 0; d < o->n(); ++d) i.c[d] = idx[d];
  return o->face_vel(i, j);
}

}  // extern "C"
