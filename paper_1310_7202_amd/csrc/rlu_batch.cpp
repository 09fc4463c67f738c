// rlu_factor_batched: Algorithm 4.1 (Shabat et al., Section 4) for many
// independent problems of different shapes, each kernel of the method
// launched once for the whole batch.
//
//   * Products (Steps 2, 5, 7) are grouped GEMMs: one launch computes the
//     tiles of every problem, listed in a table of (problem, tile) pairs.
//     Whole problems are dealt to the eight XCDs (largest first, to the
//     least loaded) and a workgroup's index decides its XCD (b mod 8), so
//     the tiles of one problem share that XCD's L2 (G in Step 2, Lv in
//     Step 5).  The tile shape of each product comes from the tuning table
//     below; the Gram product splits its long K.
//   * The two pivoted LUs (Steps 3 and 6) run as one persistent launch each:
//     every problem's panel is a "gang" of workgroups that exchange pivots,
//     gangs are packed into rounds of at most the number of workgroups the
//     device holds at once (chains of equal length together, members of a
//     gang on one XCD where it fits), and each workgroup runs its members of
//     successive rounds back to back.
//   * The Gram inverses take one workgroup per 64 x 64 tile of every
//     problem and one launch per 64 pivots; the assembly of p, q, U, L_b
//     and info is one launch.
// The launch sequence is captured once into a HIP graph and replayed while
// the same problems and buffers come back; the task tables live in the
// handle's batch workspace and are uploaded only when the batch changes.
#include "rlu_internal.h"
#include "tuned_tiles.h"

#include <algorithm>
#include <array>
#include <cstring>
#include <numeric>
#include <vector>

namespace {

using namespace rlu;
using namespace rlu_detail;

struct Item {
  rlu_problem_t pb;
  rlu_buffers_t io;
  size_t G = 0, Y = 0, S = 0, gj = 0, part = 0, C = 0, Bst = 0, Lb = 0;
  size_t pos_y = 0, rstep_y = 0, piv_y = 0, ipiv_y = 0;
  size_t pos_b = 0, rstep_b = 0, piv_b = 0, ipiv_b = 0;
  size_t flags = 0, xy = 0, xb = 0, xz = 0;  // cleared before each run
  size_t zt = 0, gz = 0, piv_z = 0, ipiv_z = 0;  // power iterations (Section 5.2)
  int gram_ks = 1;
  int nwg_y = 0, R_y = 0, nwg_b = 0, R_b = 0, nwg_z = 0, R_z = 0;
};

// The four panel runs: Step 3 on Y, Step 6 on B^T, and the two
// normalizations of the power iterations, on Y (zero pivots recorded apart
// from Step 3's) and on Z^T (n x l, stored l x n like B^T).
enum class PanelRun { Y, BT, YNorm, Z };

struct GemmLaunch {
  int cfg = 0;
  bool lp = false;
  size_t tasks = 0, map = 0;  // table offsets
  int ntasks = 0, nwg = 0;
};

struct PanelLaunch {
  size_t tasks = 0, sched = 0;
  int rounds = 0, nslots = 0, maxR = 0;
  size_t lds = 0;
};

struct Plan {
  std::vector<Item> items;
  int tile[5] = {-1, -1, -1, -1, -1};  // per-product overrides of the tile table
  bool lp = false, fp16 = false, f32 = false;
  size_t zero_bytes = 0;  // [0, zero_bytes) of the workspace: flags and exchange areas
  size_t data_end = 0;
  size_t tab_off = 0;     // tables start here
  size_t total = 0;
  std::vector<char> tab;  // host image of the tables
  // launches
  size_t gauss = 0; int n_gauss = 0; int64_t gauss_max = 0;
  size_t absmax = 0;  // FP16: max|A| of each problem into int 8 of its flags
  size_t fin = 0; int n_fin = 0; int64_t fin_max = 0;  // non-finite checks of the sketches
  std::vector<GemmLaunch> sketch, gram, project, solve, forml;
  size_t gram_all = 0; int gram_count = 0; int64_t gram_max = 0; bool gram_split = false;
  PanelLaunch py, pbt;
  // power iterations: q rounds of panel(Y), Z^T = Lv^T A, panel(Z), the
  // dense Lv(Z), Y = A Lv(Z); the exchange areas are cleared before each run
  int power = 0;
  size_t xch_begin = 0;   // [xch_begin, zero_bytes): the exchange areas
  std::vector<GemmLaunch> zproj, resketch;
  PanelLaunch pyn, pz;
  size_t lvd = 0; int64_t lvd_max = 0;
  size_t spd = 0; int64_t kmax = 0;
  size_t asmb = 0; int64_t asm_max = 0;
};

// Rows per workgroup of a panel: the most (at most 512, at least 64) whose
// LDS image fits for a panel of that width, together with the margin
// plan_panels adds for a launch compiled for 512 rows.  The panel kernel
// takes any row count up to its compiled one, so the count need not be a
// power of two: fewer workgroups per panel means fewer rounds of the batched
// launch.  A panel too wide for 64 rows (more than 294 columns) makes the
// batch unsupported (the server runs such a request alone).
constexpr size_t kPanelLdsBudget = 159 * 1024;

int panel_rows_for(int ncols) {
  if (ncols < 1) return 0;
  // the largest r with panel_lds_bytes(r, c) = 8 (r c + 5 c + r) and the
  // margin 8 ((c - 1) r + 512) both within the budget
  const int64_t b8 = (int64_t)(kPanelLdsBudget / 8), c = ncols;
  int64_t r = 512;
  r = std::min(r, b8 >= 5 * c ? (b8 - 5 * c) / (c + 1) : 0);
  if (c > 1) r = std::min(r, (b8 - 512) / (c - 1));
  if (r < 64) return 0;
  // the closed form restates panel_lds_bytes; keep the two in step
  if (panel_lds_bytes((int)r, ncols) > kPanelLdsBudget) return 0;
  return (int)r;
}

// Tile shape of a grouped product: a handle override, else the tuned table,
// else the built-in rule (the sketch takes a tile at least as wide as its
// output, so each tile row of A is read once; the others 64 x 64).
int pick_cfg(const Plan& P, GemmRole role, int64_t N) {
  const int r = (int)role;
  if (P.tile[r] >= 0) return P.tile[r];
  const int t = tuned::kGroupedTile[r][P.f32 ? 1 : 0];
  if (t >= 0 && gemm_group_cfg_valid(t)) return t;
  if (role == GemmRole::Sketch) {
    if (N <= 64) return GEMM_CFG_64x64;
    if (N <= 112) return GEMM_CFG_64x112;
  }
  return GEMM_CFG_64x64;
}

// Gram product S = Lv^T Lv has a k x k output and K = m: split K so that a
// problem's tiles are at most 512 deep.
int gram_split_for(int64_t m) {
  int ks = 1;
  while (ks < 16 && m / (2 * ks) >= 512) ks *= 2;
  return ks;
}

class TableWriter {
 public:
  explicit TableWriter(std::vector<char>& buf) : buf_(buf) {}
  template <typename T>
  size_t put(const std::vector<T>& v) {
    const size_t off = align_up(buf_.size(), 64);
    buf_.resize(off + std::max<size_t>(v.size() * sizeof(T), 1));
    if (!v.empty()) std::memcpy(buf_.data() + off, v.data(), v.size() * sizeof(T));
    return off;
  }
 private:
  std::vector<char>& buf_;
};

// Deal whole tasks to the 8 XCDs (largest first, least loaded XCD) and lay
// the tiles out so that workgroup b, which runs on XCD b % 8, takes the next
// tile of its XCD.  Padding entries have task -1.
std::vector<int2> xcd_map(const std::vector<int>& ntiles, const std::vector<int>& task_id) {
  std::vector<int> order(ntiles.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return ntiles[a] > ntiles[b]; });
  std::array<std::vector<int2>, 8> lists;
  std::array<long long, 8> load{};
  for (int t : order) {
    int x = 0;
    for (int c = 1; c < 8; ++c)
      if (load[c] < load[x]) x = c;
    for (int i = 0; i < ntiles[t]; ++i) lists[x].push_back(int2{task_id[t], i});
    load[x] += ntiles[t];
  }
  size_t len = 0;
  for (auto& l : lists) len = std::max(len, l.size());
  std::vector<int2> map(8 * len, int2{-1, 0});
  for (int x = 0; x < 8; ++x)
    for (size_t i = 0; i < lists[x].size(); ++i) map[x + 8 * i] = lists[x][i];
  return map;
}

// Build the grouped launches of one product: tasks[i] with their tile shape
// cfg[i]; one launch per distinct shape.
void add_gemm_launches(TableWriter& tw, std::vector<GemmTaskDev> tasks, const std::vector<int>& cfg,
                       bool lp, std::vector<GemmLaunch>& out) {
  std::vector<int> shapes(cfg);
  std::sort(shapes.begin(), shapes.end());
  shapes.erase(std::unique(shapes.begin(), shapes.end()), shapes.end());
  for (int c : shapes) {
    std::vector<GemmTaskDev> sel;
    std::vector<int> ntiles, ids;
    for (size_t i = 0; i < tasks.size(); ++i) {
      if (cfg[i] != c) continue;
      GemmTaskDev t = tasks[i];
      int bm, bn;
      gemm_group_tile(c, &bm, &bn);
      t.tiles_m = (int)((t.M + bm - 1) / bm);
      t.tiles_n = (int)((t.N + bn - 1) / bn);
      if (t.M <= 0 || t.N <= 0) continue;
      ids.push_back((int)sel.size());
      ntiles.push_back(t.tiles_m * t.tiles_n * std::max(1, t.ksplit));
      sel.push_back(t);
    }
    if (sel.empty()) continue;
    GemmLaunch L;
    L.cfg = c;
    L.lp = lp;
    L.ntasks = (int)sel.size();
    std::vector<int2> map = xcd_map(ntiles, ids);
    L.nwg = (int)map.size();
    L.tasks = tw.put(sel);
    L.map = tw.put(map);
    out.push_back(L);
  }
}

// Pack gangs (one per panel) into rounds of nslots workgroups.  Longer
// chains first; a gang goes to the first round with room, on one XCD if one
// has enough free slots (the fullest such XCD), else spread over XCDs.
int schedule_gangs(const std::vector<int>& nwg, const std::vector<int>& ncols, int nslots,
                   std::vector<int>& sched) {
  std::vector<int> order(nwg.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return ncols[a] != ncols[b] ? ncols[a] > ncols[b] : nwg[a] > nwg[b];
  });
  typedef std::array<std::vector<int>, 8> Free;
  std::vector<Free> rounds;
  std::vector<std::vector<int>> entries;  // per round: slot -> entry
  auto new_round = [&]() {
    Free f;
    for (int b = nslots - 1; b >= 0; --b) f[b % 8].push_back(b);  // pop_back gives lowest
    rounds.push_back(f);
    entries.push_back(std::vector<int>(nslots, -1));
  };
  for (int t : order) {
    const int need = nwg[t];
    for (size_t r = 0;; ++r) {
      if (r == rounds.size()) new_round();
      Free& f = rounds[r];
      int total = 0, best = -1;
      for (int x = 0; x < 8; ++x) {
        total += (int)f[x].size();
        if ((int)f[x].size() >= need && (best < 0 || f[x].size() < f[best].size())) best = x;
      }
      if (total < need) continue;
      std::vector<int> slots;
      if (best >= 0) {
        for (int i = 0; i < need; ++i) { slots.push_back(f[best].back()); f[best].pop_back(); }
      } else {
        while ((int)slots.size() < need) {
          int x = 0;
          for (int c = 1; c < 8; ++c)
            if (f[c].size() > f[x].size()) x = c;
          slots.push_back(f[x].back());
          f[x].pop_back();
        }
      }
      for (int i = 0; i < need; ++i) entries[r][slots[i]] = (t << 8) | i;
      break;
    }
  }
  sched.clear();
  for (auto& e : entries) sched.insert(sched.end(), e.begin(), e.end());
  return (int)rounds.size();
}

// The workspace base the task tables point into; null while the tables are
// only being sized, when the addresses they hold are placeholders (a
// non-null constant plus the offset, never dereferenced) rather than
// arithmetic on a null pointer.
struct WsBase {
  char* p;
  char* operator+(size_t off) const {
    return p ? p + off : reinterpret_cast<char*>(uintptr_t{4096} + off);
  }
  bool operator==(std::nullptr_t) const { return p == nullptr; }
};

rlu_status_t plan_panels(const Plan& P, PanelRun run, int cus, WsBase base, TableWriter& tw,
                         PanelLaunch& L) {
  const bool second = run == PanelRun::BT;
  const bool zrun = run == PanelRun::Z;
  // every problem keeps its own rows per workgroup (the most its width
  // allows); the launch is compiled for the largest and sized for the
  // largest LDS image, including the bulk update's read of a full 64 * RPL
  // rows past the last column of a shorter block
  int R = 0;
  size_t lds = 0;
  for (const Item& it : P.items) R = std::max(R, second ? it.R_b : zrun ? it.R_z : it.R_y);
  if (R == 0) return RLU_ERR_UNSUPPORTED;
  const int rmax = R <= 64 ? 64 : R <= 128 ? 128 : R <= 256 ? 256 : 512;
  for (const Item& it : P.items) {
    const int r = second ? it.R_b : zrun ? it.R_z : it.R_y;
    const int c = (int)(second ? it.pb.k : it.pb.l);
    lds = std::max(lds, panel_lds_bytes(r, c));
    lds = std::max(lds, (size_t)8 * ((size_t)(c - 1) * r + rmax));
  }
  if (lds > kPanelLdsBudget) return RLU_ERR_UNSUPPORTED;
  // Sizing pass (no base): no device query; at least one workgroup per CU
  // is resident and at most four (512-thread workgroups), which bounds the
  // schedule's size from above.
  const bool sizing = base == nullptr;
  int slots = sizing ? cus : panel_batched_slots(R, lds, cus);
  if (slots <= 0) return RLU_ERR_DEVICE;
  if (slots > 4 * cus) slots = 4 * cus;
  std::vector<PanelTaskDev> tasks;
  std::vector<int> nwg, ncols;
  for (const Item& it : P.items) {
    PanelTaskDev t{};
    if (zrun) {
      t.X = (double*)(base + it.zt); t.rs = it.pb.l; t.cs = 1;
      t.nrows = (int)it.pb.n; t.ncols = (int)it.pb.l;
      t.nwg = it.nwg_z; t.R = it.R_z;
      t.pos = (int*)(base + it.pos_b); t.rstep = (int*)(base + it.rstep_b);
      t.piv_row = (int*)(base + it.piv_z); t.ipiv = (int*)(base + it.ipiv_z);
      t.info = (int*)(base + it.flags) + 3;
      t.xch = base + it.xz;
    } else if (!second) {
      t.X = (double*)(base + it.Y); t.rs = 1; t.cs = it.pb.m;
      t.nrows = (int)it.pb.m; t.ncols = (int)it.pb.l;
      t.nwg = it.nwg_y; t.R = it.R_y;
      t.pos = (int*)(base + it.pos_y); t.rstep = (int*)(base + it.rstep_y);
      t.piv_row = (int*)(base + it.piv_y); t.ipiv = (int*)(base + it.ipiv_y);
      t.info = (int*)(base + it.flags) + (run == PanelRun::YNorm ? 3 : 0);
      t.xch = base + it.xy;
    } else {
      t.X = (double*)(base + it.Bst); t.rs = it.pb.k; t.cs = 1;
      t.nrows = (int)it.pb.n; t.ncols = (int)it.pb.k;
      t.nwg = it.nwg_b; t.R = it.R_b;
      t.pos = (int*)(base + it.pos_b); t.rstep = (int*)(base + it.rstep_b);
      t.piv_row = (int*)(base + it.piv_b); t.ipiv = (int*)(base + it.ipiv_b);
      t.info = (int*)(base + it.flags) + 1;
      t.xch = base + it.xb;
    }
    t.fail = (int*)(base + it.flags) + 2;
    t.rec_stride = panel_rec_stride(t.ncols);
    if (t.nwg > slots || t.nwg > 255) return RLU_ERR_UNSUPPORTED;
    tasks.push_back(t);
    nwg.push_back(t.nwg);
    ncols.push_back(t.ncols);
  }
  std::vector<int> sched;
  if (sizing) {
    L.rounds = (int)tasks.size();
    L.nslots = 4 * cus;
    sched.assign((size_t)L.rounds * L.nslots, -1);
  } else {
    L.rounds = schedule_gangs(nwg, ncols, slots, sched);
    L.nslots = slots;
  }
  L.maxR = R;
  L.lds = lds;
  L.tasks = tw.put(tasks);
  L.sched = tw.put(sched);
  return RLU_OK;
}

// Data layout (no device addresses needed) and panel shapes.
rlu_status_t plan_layout(Plan& P, int count, const rlu_problem_t* pbs, const rlu_buffers_t* ios) {
  P.items.resize(count);
  const rlu_precision_t prec = pbs[0].precision;
  P.lp = prec == RLU_PREC_MIXED_BF16 || prec == RLU_PREC_MIXED_FP16;
  P.fp16 = prec == RLU_PREC_MIXED_FP16;
  P.f32 = pbs[0].dtype == RLU_F32;
  size_t off = 0;
  auto take = [&](size_t& slot, size_t bytes) {
    slot = off;
    off = align_up(off + std::max<size_t>(bytes, 1));
  };
  P.power = pbs[0].power_iters;
  // cleared region first: the flags of every problem, then the exchange
  // areas (which the power iterations clear again before each panel run)
  for (int i = 0; i < count; ++i) {
    Item& it = P.items[i];
    it.pb = pbs[i];
    it.io = ios[i];
    const rlu_problem_t& pb = it.pb;
    const int Ry = panel_rows_for((int)pb.l), Rb = panel_rows_for((int)pb.k);
    if (Ry == 0 || Rb == 0) return RLU_ERR_UNSUPPORTED;
    it.nwg_y = (int)((pb.m + Ry - 1) / Ry);
    it.R_y = (int)((pb.m + it.nwg_y - 1) / it.nwg_y);
    it.nwg_b = (int)((pb.n + Rb - 1) / Rb);
    it.R_b = (int)((pb.n + it.nwg_b - 1) / it.nwg_b);
    if (P.power > 0) {
      it.nwg_z = (int)((pb.n + Ry - 1) / Ry);
      it.R_z = (int)((pb.n + it.nwg_z - 1) / it.nwg_z);
    }
    take(it.flags, 64);
  }
  P.xch_begin = off;
  for (int i = 0; i < count; ++i) {
    Item& it = P.items[i];
    const rlu_problem_t& pb = it.pb;
    take(it.xy, it.nwg_y > 1 ? panel_xch_bytes(it.nwg_y, (int)pb.l) : 0);
    take(it.xb, it.nwg_b > 1 ? panel_xch_bytes(it.nwg_b, (int)pb.k) : 0);
    take(it.xz, it.nwg_z > 1 ? panel_xch_bytes(it.nwg_z, (int)pb.l) : 0);
  }
  P.zero_bytes = off;
  const size_t d = sizeof(double);
  for (int i = 0; i < count; ++i) {
    Item& it = P.items[i];
    const int64_t m = it.pb.m, n = it.pb.n, k = it.pb.k, l = it.pb.l;
    const size_t sa = it.pb.dtype == RLU_F32 ? sizeof(float) : sizeof(double);
    take(it.G, it.pb.G ? 0 : (size_t)n * l * sa);
    take(it.Y, (size_t)m * l * d);
    it.gram_ks = gram_split_for(m);
    take(it.part, it.gram_ks > 1 ? (size_t)it.gram_ks * k * k * d : 0);
    take(it.S, (size_t)k * k * d);
    take(it.gj, spd_inverse_scratch_elems(k) * d);
    take(it.C, (size_t)k * n * d);
    take(it.Bst, (size_t)k * n * d);
    take(it.Lb, (size_t)k * k * d);
    take(it.pos_y, (size_t)m * 4);
    take(it.rstep_y, (size_t)m * 4);
    take(it.piv_y, (size_t)l * 4);
    take(it.ipiv_y, (size_t)l * 4);
    take(it.pos_b, (size_t)n * 4);
    take(it.rstep_b, (size_t)n * 4);
    take(it.piv_b, (size_t)k * 4);
    take(it.ipiv_b, (size_t)k * 4);
    const bool pw = P.power > 0;
    take(it.zt, pw ? (size_t)l * n * d : 0);
    take(it.gz, pw ? (size_t)n * l * sa : 0);
    take(it.piv_z, pw ? (size_t)l * 4 : 0);
    take(it.ipiv_z, pw ? (size_t)l * 4 : 0);
  }
  P.data_end = off;
  P.tab_off = off;
  return RLU_OK;
}

// Task tables for the workspace at `base` (base may be null to size them).
rlu_status_t build_tables(Plan& P, WsBase base, int cus) {
  P.tab.clear();
  P.sketch.clear(); P.gram.clear(); P.project.clear(); P.solve.clear(); P.forml.clear();
  P.zproj.clear(); P.resketch.clear();
  TableWriter tw(P.tab);
  // Step 1
  std::vector<GaussTaskDev> gauss;
  P.gauss_max = 0;
  for (const Item& it : P.items) {
    if (it.pb.G) continue;
    gauss.push_back(GaussTaskDev{base + it.G, it.pb.n, it.pb.n, it.pb.l, it.pb.seed});
    P.gauss_max = std::max<int64_t>(P.gauss_max, it.pb.n * it.pb.l);
  }
  P.n_gauss = (int)gauss.size();
  P.gauss = tw.put(gauss);
  // FP16 products scale A by a power of two chosen from max|A|
  auto amax_of = [&](const Item& it) -> const unsigned* {
    return P.fp16 ? (const unsigned*)(base + it.flags) + 8 : nullptr;
  };
  if (P.fp16) {
    std::vector<AbsmaxTaskDev> am;
    for (const Item& it : P.items)
      am.push_back(AbsmaxTaskDev{(const float*)it.io.A, it.io.lda, it.pb.m, it.pb.n,
                                 (unsigned*)(base + it.flags) + 8});
    P.absmax = tw.put(am);
  }
  // Step 2: Y = A G
  {
    std::vector<GemmTaskDev> t;
    std::vector<int> cfg;
    for (const Item& it : P.items) {
      GemmTaskDev g{};
      g.M = it.pb.m; g.N = it.pb.l; g.K = it.pb.n;
      g.A = it.io.A; g.lda = it.io.lda;
      g.B = it.pb.G ? it.pb.G : (const void*)(base + it.G);
      g.ldb = it.pb.G ? it.pb.ldg : it.pb.n;
      g.C = base + it.Y; g.ldc = it.pb.m;
      g.ksplit = 1;
      g.amax = amax_of(it);
      t.push_back(g);
      cfg.push_back(P.lp ? GEMM_CFG_64x64 : pick_cfg(P, GemmRole::Sketch, g.N));
    }
    add_gemm_launches(tw, t, cfg, P.lp, P.sketch);
  }
  // the non-finite checks of the problems that ask for one (on Y = A G)
  {
    std::vector<FiniteTaskDev> fin;
    P.fin_max = 0;
    for (const Item& it : P.items) {
      if (!(it.pb.flags & RLU_FLAG_CHECK_FINITE)) continue;
      fin.push_back(FiniteTaskDev{(const double*)(base + it.Y), it.pb.m * it.pb.l,
                                  (int*)(base + it.flags) + 4});
      P.fin_max = std::max<int64_t>(P.fin_max, it.pb.m * it.pb.l);
    }
    P.n_fin = (int)fin.size();
    P.fin = tw.put(fin);
  }
  // Section 5.2: the tables of one round of the power iterations
  if (P.power > 0) {
    rlu_status_t st = plan_panels(P, PanelRun::YNorm, cus, base, tw, P.pyn);
    if (st != RLU_OK) return st;
    std::vector<GemmTaskDev> t, r;
    std::vector<int> cfg, rcfg;
    std::vector<LvDenseTaskDev> lv;
    P.lvd_max = 0;
    for (const Item& it : P.items) {
      GemmTaskDev g{};  // Z^T = Lv(Y)^T A  (l x n)
      g.M = it.pb.l; g.N = it.pb.n; g.K = it.pb.m;
      g.A = base + it.Y; g.lda = it.pb.m; g.astep = (const int*)(base + it.rstep_y);
      g.B = it.io.A; g.ldb = it.io.lda;
      g.C = base + it.zt; g.ldc = it.pb.l;
      g.ksplit = 1;
      g.amax = amax_of(it);
      t.push_back(g);
      cfg.push_back(P.lp ? GEMM_CFG_64x64 : pick_cfg(P, GemmRole::Project, g.N));
      LvDenseTaskDev x{};  // Lv(Z), n x l, in the storage type
      x.X = (const double*)(base + it.zt); x.rs = it.pb.l; x.cs = 1;
      x.rstep = (const int*)(base + it.rstep_b);
      x.out = base + it.gz; x.ldo = it.pb.n; x.rows = it.pb.n; x.cols = it.pb.l;
      lv.push_back(x);
      P.lvd_max = std::max<int64_t>(P.lvd_max, it.pb.n * it.pb.l);
      GemmTaskDev y{};  // Y = A Lv(Z)
      y.M = it.pb.m; y.N = it.pb.l; y.K = it.pb.n;
      y.A = it.io.A; y.lda = it.io.lda;
      y.B = base + it.gz; y.ldb = it.pb.n;
      y.C = base + it.Y; y.ldc = it.pb.m;
      y.ksplit = 1;
      y.amax = amax_of(it);
      r.push_back(y);
      rcfg.push_back(P.lp ? GEMM_CFG_64x64 : pick_cfg(P, GemmRole::Sketch, y.N));
    }
    add_gemm_launches(tw, t, cfg, P.lp, P.zproj);
    st = plan_panels(P, PanelRun::Z, cus, base, tw, P.pz);
    if (st != RLU_OK) return st;
    P.lvd = tw.put(lv);
    add_gemm_launches(tw, r, rcfg, P.lp, P.resketch);
  }
  // Step 3
  rlu_status_t st = plan_panels(P, PanelRun::Y, cus, base, tw, P.py);
  if (st != RLU_OK) return st;
  // Step 5: S = Lv^T Lv (split K), S <- S^{-1}, C = Lv^T A, B = S^{-1} C
  {
    std::vector<GemmTaskDev> t;
    std::vector<int> cfg;
    P.gram_max = 0;
    P.gram_split = false;
    for (const Item& it : P.items) {
      GemmTaskDev g{};
      g.M = it.pb.k; g.N = it.pb.k; g.K = it.pb.m;
      g.A = base + it.Y; g.lda = it.pb.m; g.astep = (const int*)(base + it.rstep_y);
      g.B = base + it.Y; g.ldb = it.pb.m; g.bstep = (const int*)(base + it.rstep_y);
      g.C = base + it.S; g.ldc = it.pb.k;
      g.ksplit = it.gram_ks;
      g.partial = it.gram_ks > 1 ? (void*)(base + it.part) : nullptr;
      if (it.gram_ks > 1) P.gram_split = true;
      P.gram_max = std::max<int64_t>(P.gram_max, it.pb.k * it.pb.k);
      t.push_back(g);
      cfg.push_back(pick_cfg(P, GemmRole::Gram, g.N));
    }
    add_gemm_launches(tw, t, cfg, false, P.gram);
    // all tasks again, in problem order, for the split-K sums
    for (auto& g : t) {
      g.tiles_m = g.tiles_n = 1;
    }
    P.gram_count = (int)t.size();
    P.gram_all = tw.put(t);
  }
  {
    std::vector<SpdTaskDev> spd;
    P.kmax = 0;
    for (const Item& it : P.items) {
      spd.push_back(SpdTaskDev{(double*)(base + it.S), (int)it.pb.k, (double*)(base + it.gj)});
      P.kmax = std::max<int64_t>(P.kmax, it.pb.k);
    }
    P.spd = tw.put(spd);
  }
  {
    std::vector<GemmTaskDev> t;
    std::vector<int> cfg;
    for (const Item& it : P.items) {
      GemmTaskDev g{};
      g.M = it.pb.k; g.N = it.pb.n; g.K = it.pb.m;
      g.A = base + it.Y; g.lda = it.pb.m; g.astep = (const int*)(base + it.rstep_y);
      g.B = it.io.A; g.ldb = it.io.lda;
      g.C = base + it.C; g.ldc = it.pb.k;
      g.ksplit = 1;
      g.amax = amax_of(it);
      t.push_back(g);
      cfg.push_back(P.lp ? GEMM_CFG_64x64 : pick_cfg(P, GemmRole::Project, g.N));
    }
    add_gemm_launches(tw, t, cfg, P.lp, P.project);
  }
  {
    std::vector<GemmTaskDev> t;
    std::vector<int> cfg;
    for (const Item& it : P.items) {
      GemmTaskDev g{};
      g.M = it.pb.k; g.N = it.pb.n; g.K = it.pb.k;
      g.A = base + it.S; g.lda = it.pb.k;
      g.B = base + it.C; g.ldb = it.pb.k;
      g.C = base + it.Bst; g.ldc = it.pb.k;
      g.ksplit = 1;
      t.push_back(g);
      cfg.push_back(pick_cfg(P, GemmRole::Solve, g.N));
    }
    add_gemm_launches(tw, t, cfg, false, P.solve);
  }
  // Step 6
  st = plan_panels(P, PanelRun::BT, cus, base, tw, P.pbt);
  if (st != RLU_OK) return st;
  // Steps 7-8
  {
    std::vector<AsmTaskDev> a;
    P.asm_max = 0;
    for (const Item& it : P.items) {
      AsmTaskDev x{};
      x.pos_y = (const int*)(base + it.pos_y);
      x.pos_b = (const int*)(base + it.pos_b);
      x.Bst = (const double*)(base + it.Bst);
      x.piv_b = (const int*)(base + it.piv_b);
      x.rstep_b = (const int*)(base + it.rstep_b);
      x.m = it.pb.m; x.n = it.pb.n; x.k = it.pb.k;
      x.p = it.io.p; x.q = it.io.q;
      x.U = it.io.U; x.ldu = it.io.ldu;
      x.Lb = (double*)(base + it.Lb);
      x.flags = (const int*)(base + it.flags);
      x.info = it.io.info;
      a.push_back(x);
      P.asm_max = std::max<int64_t>(P.asm_max, x.m + x.n + x.k * x.n + x.k * x.k);
    }
    P.asmb = tw.put(a);
  }
  {
    std::vector<GemmTaskDev> t;
    std::vector<int> cfg;
    for (const Item& it : P.items) {
      GemmTaskDev g{};
      g.M = it.pb.m; g.N = it.pb.k; g.K = it.pb.k;
      g.A = base + it.Y; g.lda = it.pb.m; g.astep = (const int*)(base + it.rstep_y);
      g.B = base + it.Lb; g.ldb = it.pb.k;
      g.C = it.io.L; g.ldc = it.io.ldl;
      g.rowmap = (const int*)(base + it.pos_y);
      g.ksplit = 1;
      t.push_back(g);
      cfg.push_back(pick_cfg(P, GemmRole::FormL, g.N));
    }
    add_gemm_launches(tw, t, cfg, false, P.forml);
  }
  P.total = P.tab_off + align_up(P.tab.size());
  return RLU_OK;
}

rlu_status_t enqueue_gemms(const std::vector<GemmLaunch>& ls, char* tab, GemmRole role, OpA opa,
                           bool f32, bool fp16, hipStream_t s) {
  for (const GemmLaunch& L : ls) {
    const GemmTaskDev* t = (const GemmTaskDev*)(tab + L.tasks);
    const int2* map = (const int2*)(tab + L.map);
    if (L.lp) HIP_TRY(launch_gemm_lp_grouped(opa, fp16, t, map, L.nwg, s));
    else HIP_TRY(launch_gemm_grouped_role(role, f32, L.cfg, t, map, L.nwg, s));
  }
  return RLU_OK;
}

// The launch sequence of a batch on stream s.
// Panel launches keep every workgroup of the device busy; two of them must
// never run at once (their gangs could hold each other's workgroups), so an
// optional gate event orders each panel launch after the previous one.
hipError_t gated_panel(const PanelLaunch& L, char* tab, hipEvent_t gate, long long tmo,
                       hipStream_t s) {
  if (gate) {
    hipError_t e = hipStreamWaitEvent(s, gate, 0);
    if (e != hipSuccess) return e;
  }
  hipError_t e = launch_panel_lu_batched((const PanelTaskDev*)(tab + L.tasks),
                                         (const int*)(tab + L.sched), L.rounds, L.nslots, L.maxR,
                                         L.lds, tmo, s);
  if (e == hipSuccess && gate) e = hipEventRecord(gate, s);
  return e;
}

template <typename T>
rlu_status_t enqueue(rlu_handle_s* h, const Plan& P, char* base, hipEvent_t gate, hipStream_t s) {
  char* tab = base + P.tab_off;
  const int count = (int)P.items.size();
  HIP_TRY(launch_fill_u32((uint32_t*)base, P.zero_bytes / 4, 0u, s));
  if (P.fp16)
    HIP_TRY(launch_absmax_batched((const AbsmaxTaskDev*)(tab + P.absmax), count, s));
  if (P.n_gauss > 0) {
    PhaseScope ph(h, PH_GAUSSIAN, s);
    HIP_TRY(launch_gaussian_batched<T>((const GaussTaskDev*)(tab + P.gauss), P.n_gauss,
                                       P.gauss_max, s));
  }
  {
    PhaseScope ph(h, PH_SKETCH, s);
    rlu_status_t st = enqueue_gemms(P.sketch, tab, GemmRole::Sketch, OpA::Plain, P.f32, P.fp16, s);
    if (st != RLU_OK) return st;
  }
  if (P.n_fin > 0)
    HIP_TRY(launch_check_finite_batched((const FiniteTaskDev*)(tab + P.fin), P.n_fin, P.fin_max, s));
  const long long tmo = h->xch_timeout;
  if (P.power > 0) {
    PhaseScope ph(h, PH_POWER, s);
    uint32_t* xch = (uint32_t*)(base + P.xch_begin);
    const size_t xwords = (P.zero_bytes - P.xch_begin) / 4;
    for (int r = 0; r < P.power; ++r) {
      HIP_TRY(launch_fill_u32(xch, xwords, 0u, s));
      HIP_TRY(gated_panel(P.pyn, tab, gate, tmo, s));
      rlu_status_t st = enqueue_gemms(P.zproj, tab, GemmRole::Project, OpA::LvT, P.f32, P.fp16, s);
      if (st != RLU_OK) return st;
      HIP_TRY(launch_fill_u32(xch, xwords, 0u, s));
      HIP_TRY(gated_panel(P.pz, tab, gate, tmo, s));
      HIP_TRY(launch_lv_dense_batched<T>((const LvDenseTaskDev*)(tab + P.lvd), count, P.lvd_max,
                                         s));
      st = enqueue_gemms(P.resketch, tab, GemmRole::Sketch, OpA::Plain, P.f32, P.fp16, s);
      if (st != RLU_OK) return st;
    }
    HIP_TRY(launch_fill_u32(xch, xwords, 0u, s));
  }
  {
    PhaseScope ph(h, PH_PANEL_Y, s);
    HIP_TRY(gated_panel(P.py, tab, gate, tmo, s));
  }
  {
    PhaseScope ph(h, PH_GRAM, s);
    rlu_status_t st = enqueue_gemms(P.gram, tab, GemmRole::Gram, OpA::LvT, P.f32, false, s);
    if (st != RLU_OK) return st;
    if (P.gram_split)
      HIP_TRY(launch_splitk_sum_grouped((const GemmTaskDev*)(tab + P.gram_all), P.gram_count,
                                        P.gram_max, s));
  }
  {
    PhaseScope ph(h, PH_GRAM_INV, s);
    HIP_TRY(launch_spd_inverse_batched((const SpdTaskDev*)(tab + P.spd), count, P.kmax, s));
  }
  {
    PhaseScope ph(h, PH_PROJECT, s);
    rlu_status_t st = enqueue_gemms(P.project, tab, GemmRole::Project, OpA::LvT, P.f32, P.fp16, s);
    if (st != RLU_OK) return st;
  }
  {
    PhaseScope ph(h, PH_SOLVE, s);
    rlu_status_t st = enqueue_gemms(P.solve, tab, GemmRole::Solve, OpA::Plain, P.f32, false, s);
    if (st != RLU_OK) return st;
  }
  {
    PhaseScope ph(h, PH_PANEL_B, s);
    HIP_TRY(gated_panel(P.pbt, tab, gate, tmo, s));
  }
  {
    PhaseScope ph(h, PH_ASSEMBLE, s);
    HIP_TRY(launch_assemble_batched<T>((const AsmTaskDev*)(tab + P.asmb), count, P.asm_max, s));
  }
  {
    PhaseScope ph(h, PH_FORM_L, s);
    rlu_status_t st = enqueue_gemms(P.forml, tab, GemmRole::FormL, OpA::Lv, P.f32, false, s);
    if (st != RLU_OK) return st;
  }
  return RLU_OK;
}

rlu_status_t ensure_bws(rlu_handle_s* h, size_t bytes) {
  if (bytes <= h->bws_bytes) return RLU_OK;
  // the cached graph refers to the old workspace
  if (h->bgraph.exec) { hipGraphExecDestroy(h->bgraph.exec); h->bgraph.exec = nullptr; }
  if (h->bgraph.graph) { hipGraphDestroy(h->bgraph.graph); h->bgraph.graph = nullptr; }
  h->bgraph.sig.clear();
  if (h->bws) {
    if (hipFree(h->bws) != hipSuccess) return RLU_ERR_DEVICE;
    h->bws = nullptr;
    h->bws_bytes = 0;
  }
  if (hipMalloc(&h->bws, bytes) != hipSuccess) {
    h->bws = nullptr;
    return RLU_ERR_OUT_OF_MEMORY;
  }
  h->bws_bytes = bytes;
  return RLU_OK;
}

rlu_status_t upload_tables(rlu_handle_s* h, const Plan& P, char* base, hipStream_t s) {
  const size_t bytes = P.tab.size();
  if (bytes == 0) return RLU_OK;
  HIP_TRY(hipEventSynchronize(h->ev_stage));  // the previous upload has left the stage
  if (bytes > h->stage_bytes) {
    if (h->stage) HIP_TRY(hipHostFree(h->stage));
    h->stage = nullptr;
    h->stage_bytes = 0;
    if (hipHostMalloc(&h->stage, bytes, hipHostMallocDefault) != hipSuccess) {
      h->stage = nullptr;
      return RLU_ERR_OUT_OF_MEMORY;
    }
    h->stage_bytes = bytes;
  }
  std::memcpy(h->stage, P.tab.data(), bytes);
  HIP_TRY(hipMemcpyAsync(base + P.tab_off, h->stage, bytes, hipMemcpyHostToDevice, s));
  HIP_TRY(hipEventRecord(h->ev_stage, s));
  return RLU_OK;
}

void drop_graph(rlu_handle_s* h) {
  if (h->bgraph.exec) hipGraphExecDestroy(h->bgraph.exec);
  if (h->bgraph.graph) hipGraphDestroy(h->bgraph.graph);
  h->bgraph.exec = nullptr;
  h->bgraph.graph = nullptr;
  h->bgraph.sig.clear();
}

template <typename T>
rlu_status_t capture(rlu_handle_s* h, const Plan& P) {
  // created on first use, so that handles that never batch hold no extra
  // stream (streams beyond the device's hardware queues share queues)
  if (!h->cap) HIP_TRY(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
  HIP_TRY(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
  rlu_status_t st = enqueue<T>(h, P, (char*)h->bws, nullptr, h->cap);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(h->cap, &g);
  if (st != RLU_OK || e != hipSuccess || !g) {
    if (g) hipGraphDestroy(g);
    return st != RLU_OK ? st : RLU_ERR_DEVICE;
  }
  hipGraphExec_t x = nullptr;
  if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
    hipGraphDestroy(g);
    return RLU_ERR_DEVICE;
  }
  h->bgraph.graph = g;
  h->bgraph.exec = x;
  return RLU_OK;
}

std::vector<char> signature(rlu_handle_s* h, int count, const rlu_problem_t* pbs,
                            const rlu_buffers_t* ios) {
  std::vector<char> sig(sizeof(int) + sizeof(void*) + sizeof(int) + sizeof(h->tile_override) +
                        sizeof(long long) +
                        count * (sizeof(rlu_problem_t) + sizeof(rlu_buffers_t)));
  char* p = sig.data();
  std::memcpy(p, h->tile_override, sizeof(h->tile_override)); p += sizeof(h->tile_override);
  std::memcpy(p, &h->xch_timeout, sizeof(long long)); p += sizeof(long long);
  std::memcpy(p, &count, sizeof(int)); p += sizeof(int);
  std::memcpy(p, &h->bws, sizeof(void*)); p += sizeof(void*);
  std::memcpy(p, &h->cus, sizeof(int)); p += sizeof(int);
  std::memcpy(p, pbs, count * sizeof(rlu_problem_t)); p += count * sizeof(rlu_problem_t);
  std::memcpy(p, ios, count * sizeof(rlu_buffers_t));
  return sig;
}

}  // namespace

extern "C" rlu_status_t rlu_factor_batched(rlu_handle_t h, int32_t count,
                                           const rlu_problem_t* pbs, const rlu_buffers_t* ios,
                                           rlu_stream_t stream) {
  if (!h || count < 0 || (count > 0 && (!pbs || !ios))) return RLU_ERR_INVALID_ARG;
  if (count == 0) return RLU_OK;
  {
    rlu_status_t st = batched_validate(count, pbs, ios);
    if (st != RLU_OK) return st;
  }
  DeviceScope dev(h->device);
  if (!dev.ok) return RLU_ERR_DEVICE;
  hipStream_t s = (hipStream_t)stream;

  Plan P;
  for (int r = 0; r < 5; ++r) P.tile[r] = h->tile_override[r];
  rlu_status_t st = plan_layout(P, count, pbs, ios);
  if (st != RLU_OK) return st;
  st = build_tables(P, WsBase{nullptr}, h->cus);  // sizes only
  if (st != RLU_OK) return st;
  st = ensure_bws(h, P.total);
  if (st != RLU_OK) return st;

  const bool f32 = pbs[0].dtype == RLU_F32;
  if (!h->timing) {
    std::vector<char> sig = signature(h, count, pbs, ios);
    if (h->bgraph.exec && sig == h->bgraph.sig) {
      HIP_TRY(hipGraphLaunch(h->bgraph.exec, s));
      return RLU_OK;
    }
    drop_graph(h);
    st = build_tables(P, WsBase{(char*)h->bws}, h->cus);
    if (st != RLU_OK) return st;
    if (P.total > h->bws_bytes) return RLU_ERR_DEVICE;  // the sizing pass bounds it
    st = upload_tables(h, P, (char*)h->bws, s);
    if (st != RLU_OK) return st;
    st = f32 ? capture<float>(h, P) : capture<double>(h, P);
    if (st != RLU_OK) return st;
    h->bgraph.sig = std::move(sig);
    HIP_TRY(hipGraphLaunch(h->bgraph.exec, s));
    return RLU_OK;
  }
  // timed calls run the same sequence eagerly, with phase events
  drop_graph(h);
  st = build_tables(P, WsBase{(char*)h->bws}, h->cus);
  if (st != RLU_OK) return st;
  if (P.total > h->bws_bytes) return RLU_ERR_DEVICE;  // the sizing pass bounds it
  st = upload_tables(h, P, (char*)h->bws, s);
  if (st != RLU_OK) return st;
  st = begin_timing(h);
  if (st != RLU_OK) return st;
  return f32 ? enqueue<float>(h, P, (char*)h->bws, h->ev_panel, s)
             : enqueue<double>(h, P, (char*)h->bws, h->ev_panel, s);
}

namespace rlu_detail {

// Validation shared with the server: every problem valid, one dtype and
// precision, no diagnostics.
rlu_status_t batched_validate(int count, const rlu_problem_t* pbs, const rlu_buffers_t* ios) {
  for (int i = 0; i < count; ++i) {
    rlu_status_t st = validate(&pbs[i]);
    if (st != RLU_OK) return st;
    if (ios) {
      st = validate_io(&pbs[i], &ios[i]);
      if (st != RLU_OK) return st;
    }
    if (pbs[i].flags & RLU_FLAG_DIAGNOSTICS) return RLU_ERR_INVALID_ARG;
    if (pbs[i].flags & (RLU_FLAG_RRLU | RLU_FLAG_FAST)) return RLU_ERR_UNSUPPORTED;
    if (pbs[i].power_iters != pbs[0].power_iters) return RLU_ERR_INVALID_ARG;
    if (pbs[i].dtype != pbs[0].dtype || pbs[i].precision != pbs[0].precision)
      return RLU_ERR_INVALID_ARG;
  }
  return RLU_OK;
}

// Upper bound of the batch workspace one problem adds (its data, exchange
// areas and its share of the task tables), independent of the rest of the
// batch.  Also checks that the problem fits the batched kernels.
rlu_status_t batched_item_bytes(const rlu_problem_t& pb, int cus, size_t* bytes) {
  rlu_buffers_t io{};
  io.lda = pb.m; io.ldl = pb.m; io.ldu = pb.k;
  Plan P;
  rlu_status_t st = plan_layout(P, 1, &pb, &io);
  if (st != RLU_OK) return st;
  st = build_tables(P, WsBase{nullptr}, cus);
  if (st != RLU_OK) return st;
  // in a larger batch the same entries, plus alignment and the XCD padding of
  // each tile map (< 8 entries per launch); the sizing pass already reserves
  // a full schedule row of 4 x cus slots per problem and panel
  const size_t slack = 8 * 8 * 8 + 16 * 64;
  *bytes = P.total + slack;
  return RLU_OK;
}

// Workspace a batch needs (for a caller-provided workspace).
rlu_status_t batched_ws_bytes(int count, const rlu_problem_t* pbs, const rlu_buffers_t* ios,
                              int cus, size_t* bytes) {
  Plan P;
  rlu_status_t st = plan_layout(P, count, pbs, ios);
  if (st != RLU_OK) return st;
  st = build_tables(P, WsBase{nullptr}, cus);
  if (st != RLU_OK) return st;
  *bytes = P.total;
  return RLU_OK;
}

// Enqueue a batch on stream s in the caller's workspace (no graph), panel
// launches ordered by `gate`.
rlu_status_t batched_enqueue_ws(rlu_handle_s* h, int count, const rlu_problem_t* pbs,
                                const rlu_buffers_t* ios, hipStream_t s, void* ws,
                                size_t ws_bytes, hipEvent_t gate) {
  Plan P;
  rlu_status_t st = plan_layout(P, count, pbs, ios);
  if (st != RLU_OK) return st;
  st = build_tables(P, WsBase{(char*)ws}, h->cus);
  if (st != RLU_OK) return st;
  if (P.total > ws_bytes) return RLU_ERR_INVALID_ARG;
  st = upload_tables(h, P, (char*)ws, s);
  if (st != RLU_OK) return st;
  h->cur = nullptr;
  return pbs[0].dtype == RLU_F32 ? enqueue<float>(h, P, (char*)ws, gate, s)
                                 : enqueue<double>(h, P, (char*)ws, gate, s);
}

}  // namespace rlu_detail

extern "C" rlu_status_t rlu_set_tile(rlu_handle_t h, int32_t product, int32_t cfg) {
  if (!h || product < 0 || product >= 5) return RLU_ERR_INVALID_ARG;
  if (cfg != -1 && !gemm_group_cfg_valid(cfg)) return RLU_ERR_INVALID_ARG;
  h->tile_override[product] = cfg;
  return RLU_OK;
}

extern "C" const char* rlu_tile_name(int32_t cfg) {
  return gemm_group_cfg_valid(cfg) ? gemm_cfg_name(cfg) : nullptr;
}
