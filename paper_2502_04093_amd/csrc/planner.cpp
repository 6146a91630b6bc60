// Loading planner: the error bound of a partial load (Thm. 1) and the two
// knapsack dynamic programs of Sec. 5.2 (least data for an error bound) and
// Sec. 5.3 (least error for a byte budget).
//
// Readings used:
//  * Groups are passes (one per level and dimension).  Loss delta_s of pass s
//    reaches the final reconstruction through at most S - s later predictions,
//    each of infinity norm p (1 linear, 1.25 cubic): A_s = p^(S - s).
//  * delta_s(b) = errq[s][b] * T(2 eb), errq being the exact max code loss.
//  * Rounding of a reconstruction computed in the field's dtype from truncated
//    codes: each lossy pass s is charged T_s * r with T_s = sum_{s'>=s} A_s'
//    and r = 14 u M (u unit roundoff, M bounds the magnitudes: maxabs + E in
//    error-bound mode; maxabs while planning a bitrate, 2 (maxabs + B0) when
//    reporting its bound).
//  * Error budget in 1024 units of (E - eb); cost floor(term / unit) + 1 for a
//    non-zero term.  Byte budget in at most 1024 units, costs rounded up.  Ties
//    go to the smallest number of discarded planes, last pass first.
//  * Variant (the paper's grouping, Sec. 4.3): with IPC_TARGET_LEVEL_GROUPS
//    every pass of a level discards the same number of planes; the programs
//    then choose one b per level, a level's term and bytes being the sums over
//    its passes.  The bound stays the per-pass one above.
#include "ipc_internal.h"

#include <cmath>
#include <limits>

namespace ipc {

static constexpr int G_UNITS = 1024;

static double rounding_step(const PlanTables &t, double M) { return 14.0 * t.unit_roundoff * M; }

static double term(const PlanTables &t, int s, int b, double r) {
  double v = (double(t.errq[size_t(s) * 33 + b]) * t.two_eb) * t.amp[s];
  if (b > 0) v = v + t.tail[s] * r;
  return v;
}

double plan_bound(const PlanTables &t, const std::vector<int> &plan, double M) {
  double r = rounding_step(t, M);
  double tot = t.eb;
  for (int s = 0; s < t.P; ++s)
    if (t.progressive[s]) tot = tot + term(t, s, plan[s], r);
  return tot;
}

int64_t plan_loaded(const PlanTables &t, const std::vector<int> &plan) {
  int64_t tot = t.fixed_bytes;
  for (int s = 0; s < t.P; ++s)
    if (t.progressive[s])
      for (int k = plan[s]; k < 32; ++k) tot += t.sizes[size_t(s) * 32 + k];
  return tot;
}

// passes sharing one choice, in stream order: each pass alone, or the
// anchors alone and then one group per level
static std::vector<std::vector<int>> plan_groups(const PlanTables &t, bool per_level) {
  std::vector<std::vector<int>> g;
  for (int s = 0; s < t.P; ++s) {
    if (per_level && s > 1 && t.level[s] == t.level[s - 1])
      g.back().push_back(s);
    else
      g.push_back({s});
  }
  return g;
}

static int allowed_hi(const PlanTables &t, const std::vector<int> &g, const int *limit) {
  if (!t.progressive[g[0]]) return 0;
  int hi = 32;
  if (limit)
    for (int s : g) hi = std::min(hi, limit[s]);
  return hi;
}

static double group_term(const PlanTables &t, const std::vector<int> &g, int b, double r) {
  double v = 0.0;
  for (int s : g)
    if (t.progressive[s]) v = v + term(t, s, b, r);
  return v;
}

// bytes of planes lo <= k < hi over the group's progressive passes
static int64_t group_bytes(const PlanTables &t, const std::vector<int> &g, int lo, int hi) {
  int64_t v = 0;
  for (int s : g)
    if (t.progressive[s])
      for (int k = lo; k < hi; ++k) v += t.sizes[size_t(s) * 32 + k];
  return v;
}

// The programs' inner steps: one choice (cost c, value v) applied to every
// budget cell, best[r] = max (error bound mode) or min (bitrate mode) of
// itself and prev[r - c] + v.  Branch-free, so the compiler vectorizes them;
// built for AVX2 as well as the baseline, picked by the CPU at load time.
__attribute__((target_clones("avx2", "default"))) static void max_shift_add(double *best,
                                                                           const double *prev,
                                                                           int n, int c, double v) {
  for (int r = c; r < n; ++r) {
    const double x = prev[r - c] + v;
    best[r] = x > best[r] ? x : best[r];
  }
}
__attribute__((target_clones("avx2", "default"))) static void min_shift_add(double *best,
                                                                           const double *prev,
                                                                           int n, int c, double v) {
  for (int r = c; r < n; ++r) {
    const double x = prev[r - c] + v;
    best[r] = x < best[r] ? x : best[r];
  }
}

// Every group's table is kept (NG x cells doubles); the backtrack recovers a
// group's choice at a cell as the smallest b whose candidate equals the
// table's value there, which is the choice the tie rule keeps (choices are
// applied in increasing b and replace only on strict improvement).  Choices
// that can never be kept are not applied: those with the cost (bytes) and the
// value of an earlier choice no better (a smaller b always wins or ties).
static PlanResult plan_eb(const PlanTables &t, double E, const int *limit, bool per_level) {
  PlanResult res;
  const int P = t.P;
  res.plan.assign(P, 0);
  double R = E - t.eb;
  if (!(R >= 0.0)) {
    res.flags = IPC_FLAG_CLAMPED_TO_EB;
    return res;
  }
  // E == eb: every discarded plane costs a positive term (at least T_s r), so
  // the program can only keep every plane; that plan without running it
  if (R == 0.0) return res;
  double r = rounding_step(t, t.maxabs + E);
  double u = R / G_UNITS;
  const int N = G_UNITS + 1;
  const std::vector<std::vector<int>> groups = plan_groups(t, per_level);
  const int NG = int(groups.size());
  // tables F_0 .. F_NG: F_0 = 0 (nothing chosen); saved bytes are integers
  // below 2^53, exact in doubles
  std::vector<double> F(size_t(NG + 1) * N, 0.0);
  std::vector<int> cost(size_t(NG) * 33, 0);
  std::vector<double> saved_of(size_t(NG) * 33, 0.0);
  std::vector<uint8_t> used(size_t(NG) * 33, 0);
  for (int gi = 0; gi < NG; ++gi) {
    const std::vector<int> &g = groups[gi];
    const double *prev = &F[size_t(gi) * N];
    double *cur = &F[size_t(gi + 1) * N];
    // b = 0 discards nothing: term 0, cost 0, nothing saved
    std::copy(prev, prev + N, cur);
    used[size_t(gi) * 33] = 1;
    int hi = allowed_hi(t, g, limit);
    int64_t saved = 0;
    // cheapest cost so far among choices saving exactly `plateau` bytes (saved
    // bytes never decrease with b)
    int64_t plateau = 0;
    int plateau_cost = 0;
    for (int b = 1; b <= hi; ++b) {
      saved += group_bytes(t, g, b - 1, b);
      double tv = group_term(t, g, b, r);
      int c;
      if (tv == 0.0) {
        c = 0;
      } else {
        double qv = u > 0.0 ? tv / u : std::numeric_limits<double>::infinity();
        c = (qv < double(G_UNITS)) ? int(std::floor(qv)) + 1 : G_UNITS + 1;
      }
      cost[size_t(gi) * 33 + b] = c;
      saved_of[size_t(gi) * 33 + b] = double(saved);
      if (c > G_UNITS) continue;
      if (saved == plateau) {
        // an earlier (smaller) b saves as much for no more cost
        if (c >= plateau_cost) continue;
        plateau_cost = c;
      } else {
        plateau = saved;
        plateau_cost = c;
      }
      used[size_t(gi) * 33 + b] = 1;
      max_shift_add(cur, prev, N, c, double(saved));
    }
  }
  int rr = G_UNITS;
  for (int gi = NG - 1; gi >= 0; --gi) {
    const double *prev = &F[size_t(gi) * N];
    const double want = F[size_t(gi + 1) * N + rr];
    int pick = 0;
    for (int b = 0; b <= 32; ++b) {
      if (!used[size_t(gi) * 33 + b]) continue;
      const int c = cost[size_t(gi) * 33 + b];
      if (c <= rr && prev[rr - c] + saved_of[size_t(gi) * 33 + b] == want) {
        pick = b;
        break;
      }
    }
    for (int s2 : groups[gi]) res.plan[s2] = pick;
    rr -= cost[size_t(gi) * 33 + pick];
  }
  return res;
}

static PlanResult plan_br(const PlanTables &t, double bitrate, const int *limit, bool per_level) {
  PlanResult res;
  const int P = t.P;
  res.plan.assign(P, 0);
  double bt = bitrate * double(t.n_points) / 8.0;
  if (bt >= double(t.total_bytes)) return res;  // everything fits
  int64_t budget = int64_t(std::floor(bt)) - t.fixed_bytes;
  if (limit) {
    std::vector<int> cur(limit, limit + P);
    if (budget < plan_loaded(t, cur) - t.fixed_bytes) {
      res.plan = cur;
      res.flags = IPC_FLAG_NOOP;
      return res;
    }
  }
  if (budget < 0) {
    for (int s = 0; s < P; ++s)
      if (t.progressive[s]) res.plan[s] = 32;
    res.flags = IPC_FLAG_BUDGET_BELOW_MIN;
    return res;
  }
  int64_t ub = std::max<int64_t>(1, (budget + G_UNITS - 1) / G_UNITS);
  int64_t cap = budget / ub;
  const int N = int(cap + 1);
  double r = rounding_step(t, t.maxabs);
  const double INF = std::numeric_limits<double>::infinity();
  const std::vector<std::vector<int>> groups = plan_groups(t, per_level);
  const int NG = int(groups.size());
  // tables F_0 .. F_NG: F_0 = 0, unreachable cells infinite
  std::vector<double> F(size_t(NG + 1) * N, INF);
  std::fill(F.begin(), F.begin() + N, 0.0);
  std::vector<int64_t> lcs(size_t(NG) * 33, 0);
  std::vector<double> tvs(size_t(NG) * 33, 0.0);
  std::vector<uint8_t> used(size_t(NG) * 33, 0);
  for (int gi = 0; gi < NG; ++gi) {
    const std::vector<int> &g = groups[gi];
    const double *prev = &F[size_t(gi) * N];
    double *cur = &F[size_t(gi + 1) * N];
    int hi = allowed_hi(t, g, limit);
    // least term so far among choices loading exactly `plateau` byte units
    // (loaded units never increase with b)
    int64_t plateau = -1;
    double plateau_tv = 0.0;
    for (int b = 0; b <= hi; ++b) {
      const int64_t lc = (group_bytes(t, g, b, 32) + ub - 1) / ub;
      const double tv = group_term(t, g, b, r);
      lcs[size_t(gi) * 33 + b] = lc;
      tvs[size_t(gi) * 33 + b] = tv;
      if (lc > cap) continue;
      if (lc == plateau) {
        // an earlier (smaller) b loads as little for no larger term
        if (tv >= plateau_tv) continue;
        plateau_tv = tv;
      } else {
        plateau = lc;
        plateau_tv = tv;
      }
      used[size_t(gi) * 33 + b] = 1;
      min_shift_add(cur, prev, N, int(lc), tv);
    }
  }
  if (!std::isfinite(F[size_t(NG) * N + cap])) {
    res.plan.assign(limit, limit + P);
    res.flags = IPC_FLAG_NOOP;
    return res;
  }
  int64_t rr = cap;
  for (int gi = NG - 1; gi >= 0; --gi) {
    const double *prev = &F[size_t(gi) * N];
    const double want = F[size_t(gi + 1) * N + rr];
    int pick = -1;
    for (int b = 0; b <= 32; ++b) {
      if (!used[size_t(gi) * 33 + b]) continue;
      const int64_t lc = lcs[size_t(gi) * 33 + b];
      if (lc <= rr && prev[rr - lc] + tvs[size_t(gi) * 33 + b] == want) {
        pick = b;
        break;
      }
    }
    if (pick < 0) pick = 0;  // not reached: the table's value came from some choice
    for (int s2 : groups[gi]) res.plan[s2] = pick;
    rr -= lcs[size_t(gi) * 33 + pick];
  }
  return res;
}

PlanResult plan_request(const PlanTables &t, int mode, double value, const int *limit) {
  PlanResult res;
  const bool per_level = (mode & IPC_TARGET_LEVEL_GROUPS) != 0;
  mode &= ~IPC_TARGET_LEVEL_GROUPS;
  if (mode == IPC_TARGET_EB) {
    res = plan_eb(t, value, limit, per_level);
    if (value < t.eb)
      res.bound = plan_bound(t, res.plan, t.maxabs);
    else
      res.bound = plan_bound(t, res.plan, t.maxabs + value);
  } else {
    res = plan_br(t, value, limit, per_level);
    double b0 = plan_bound(t, res.plan, t.maxabs);
    res.bound = plan_bound(t, res.plan, 2.0 * (t.maxabs + b0));
  }
  res.loaded = plan_loaded(t, res.plan);
  return res;
}

PlanTables plan_tables_from_sizes(const StreamMeta &m, const std::vector<uint64_t> &sizes) {
  PlanTables t;
  const Schedule &s = m.sched;
  t.P = int(s.passes.size());
  t.errq = m.errq;
  t.sizes.assign(sizes.begin(), sizes.end());
  t.progressive.assign(t.P, 1);
  t.progressive[0] = 0;
  for (const PassGeom &p : s.passes)
    if (p.index > 0 && p.level > s.K - m.nonprog_levels) t.progressive[p.index] = 0;
  double pval = m.interp == IPC_LINEAR ? 1.0 : 1.25;
  t.amp.assign(t.P, 0.0);
  t.tail.assign(t.P, 0.0);
  double a = 1.0, tt = 0.0;
  for (int s2 = t.P - 1; s2 >= 1; --s2) {
    t.amp[s2] = a;
    tt = tt + a;
    t.tail[s2] = tt;
    a = a * pval;
  }
  if (m.dtype == IPC_F32)
    t.two_eb = double(float(2.0 * m.eb));
  else
    t.two_eb = 2.0 * m.eb;
  t.eb = m.eb;
  t.unit_roundoff = m.dtype == IPC_F32 ? std::ldexp(1.0, -24) : std::ldexp(1.0, -53);
  t.maxabs = m.maxabs;
  t.n_points = s.n_points;
  t.total_bytes = int64_t(m.serialized_bytes);
  int64_t prog = 0;
  for (int s2 = 0; s2 < t.P; ++s2)
    if (t.progressive[s2])
      for (int k = 0; k < 32; ++k) prog += t.sizes[size_t(s2) * 32 + k];
  t.fixed_bytes = t.total_bytes - prog;
  t.level.assign(t.P, 0);
  for (const PassGeom &p : s.passes) t.level[p.index] = p.level;
  return t;
}

// plane sizes from the chunk masks; an entropy-coded stream charges every
// block the words it stores
PlanTables plan_tables(const StreamMeta &m) {
  const Schedule &s = m.sched;
  std::vector<uint64_t> sizes(s.passes.size() * 32, 0);
  size_t blk = 0;
  std::vector<uint32_t> cnt;
  for (const PassGeom &p : s.passes) {
    chunk_counts(p, cnt);
    for (int64_t c = 0; c < p.n_chunks; ++c) {
      uint32_t mk = m.masks[size_t(p.chunk_base + c)];
      if (!mk) continue;
      uint64_t W = uint64_t((cnt[size_t(c)] + 31) / 32);
      for (int k = 31; k >= 0; --k)
        if ((mk >> k) & 1u) {
          sizes[size_t(p.index) * 32 + k] += 4 * (m.coding ? uint64_t(m.block_words[blk]) : W);
          ++blk;
        }
    }
  }
  return plan_tables_from_sizes(m, sizes);
}

// Bound of the additive form of Alg. 2 (x_new = x_old + Delta): the reported
// bound of the new plan plus the rounding the additive form does where a fresh
// reconstruction does not -- the old reconstruction's own rounding (T_s r for
// the old plan's lossy passes), the difference field's (T_s1 r, s1 the first
// progressive pass, as if every pass were lossy) and the final addition (u M),
// with M the magnitude bound of the reported bound.
double plan_additive_bound(const PlanTables &t, const std::vector<int> &plan,
                           const std::vector<int> &old_plan, int mode, double value, double reported) {
  mode &= ~IPC_TARGET_LEVEL_GROUPS;
  double M;
  if (mode == IPC_TARGET_EB)
    M = value < t.eb ? t.maxabs : t.maxabs + value;
  else
    M = 2.0 * (t.maxabs + plan_bound(t, plan, t.maxabs));
  const double r = rounding_step(t, M);
  double a = reported;
  int first = -1;
  for (int s = 0; s < t.P; ++s) {
    if (!t.progressive[s]) continue;
    if (first < 0) first = s;
    if (old_plan[s] > 0) a = a + t.tail[s] * r;
  }
  if (first >= 0) a = a + t.tail[first] * r;
  return a + t.unit_roundoff * M;
}

}  // namespace ipc
