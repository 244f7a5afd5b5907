// Many sources in few launches: the batched path and its autotuner.
//
// Sources are grouped by tile family (the compiled tile shapes their patch
// size selects), in groups of at most kMaxBatch whose per-bin records fit
// a fixed budget.  Per group:
//   * one k_decorr launch per source writes that source's records (u', v',
//     W D) into its slot, reading the direction from the caller's device
//     source array, so a captured graph replays with new directions;
//   * one persistent contraction launch runs every (source, tile, k-slice)
//     work item of the group, items sized to cost alike, workgroup w taking
//     items w, w + G, w + 2G, ... (static, no atomics, nothing to reset);
//   * one finalise launch writes every patch of the group into P_all.
// Every launch is asynchronous on the caller's stream with no allocation,
// memset or host synchronisation, so the whole call can be captured into a
// HIP graph.
//
// Launch shapes per tile family (work items per compute unit, first-level
// accumulation run) come from a tuning table that psf_autotune writes by
// timing candidates on the caller's data; without a table, defaults apply.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "psf_host.hpp"

namespace psf {

namespace {

constexpr size_t kRecordBudget = size_t(16) << 30;  // bytes of per-bin records per group
constexpr int kComputeUnits = 256;                  // MI355X: one contraction workgroup per CU
constexpr int kDefaultItemsPerCU = 2;
const int kFlushCandidates[] = {32, 64, 128};
const int kItemsCandidates[] = {1, 2, 3, 4};
constexpr int kMaxItemsPerCU = 4;  // the largest candidate: bounds the workspace

// Tile family and form (general or symmetric) of a source: the sources of
// one contraction launch share both.
struct Family {
  int tbi0, tbi1, tbj0, tbj1, sym;
  bool operator==(const Family& o) const {
    return tbi0 == o.tbi0 && tbi1 == o.tbi1 && tbj0 == o.tbj0 && tbj1 == o.tbj1 && sym == o.sym;
  }
};

Family family_of(const psf_src& s) {
  TilePlan t;
  plan_tiles((s.nl + 15) / 16, (s.nm + 15) / 16, &t);
  return {t.tbi[0], t.tbi[1], t.tbj[0], t.tbj[1], sym_source(&s) ? 1 : 0};
}

struct Tuning {
  Family fam;
  int items_per_cu;
  int flush;
};

// Reads the table psf_autotune writes: a JSON object whose "families" array
// holds objects with integer fields tbi0, tbi1, tbj0, tbj1, items_per_cu,
// flush and (optional, default 0) sym.  Only that shape is accepted.
int parse_tuning(const char* json, std::vector<Tuning>* out) {
  out->clear();
  if (json == nullptr) return PSF_OK;
  const char* p = std::strstr(json, "\"families\"");
  if (p == nullptr) return fail(PSF_EINVAL, "tuning table has no \"families\"");
  p = std::strchr(p, '[');
  if (p == nullptr) return fail(PSF_EINVAL, "tuning table: \"families\" is not an array");
  const char* end = std::strchr(p, ']');
  if (end == nullptr) return fail(PSF_EINVAL, "tuning table: unterminated array");
  auto field = [](const char* obj, const char* obj_end, const char* name, int* v) {
    std::string key = std::string("\"") + name + "\"";
    const char* q = std::strstr(obj, key.c_str());
    if (q == nullptr || q > obj_end) return false;
    q = std::strchr(q + key.size(), ':');
    if (q == nullptr || q > obj_end) return false;
    return std::sscanf(q + 1, "%d", v) == 1;
  };
  for (const char* o = std::strchr(p, '{'); o != nullptr && o < end; o = std::strchr(o + 1, '{')) {
    const char* oe = std::strchr(o, '}');
    if (oe == nullptr || oe > end) return fail(PSF_EINVAL, "tuning table: unterminated entry");
    Tuning t;
    if (!field(o, oe, "tbi0", &t.fam.tbi0) || !field(o, oe, "tbi1", &t.fam.tbi1) ||
        !field(o, oe, "tbj0", &t.fam.tbj0) || !field(o, oe, "tbj1", &t.fam.tbj1) ||
        !field(o, oe, "items_per_cu", &t.items_per_cu) || !field(o, oe, "flush", &t.flush))
      return fail(PSF_EINVAL, "tuning table: entry lacks a field");
    if (!field(o, oe, "sym", &t.fam.sym)) t.fam.sym = 0;
    if (t.items_per_cu < 1 || t.items_per_cu > kMaxItemsPerCU || t.flush < 1 || t.flush > 4096)
      return fail(PSF_EINVAL, "tuning table: items_per_cu (1..%d) or flush (1..4096) out of range", kMaxItemsPerCU);
    out->push_back(t);
  }
  return PSF_OK;
}

// Work items per CU when the caller gives no table (kp: the precision the
// contraction runs in): one for the 257- and 129-pixel families, whose
// items are large, in the forms that run one workgroup per CU; four for the
// 65-pixel family, whose kernel runs two workgroups per CU (two items each);
// in the stochastic form, which runs two workgroups per CU for every
// family, two for the 257-pixel family and four for the 129-pixel one; two
// otherwise.
int default_items_per_cu(const Family& f, int kp) {
  if (f.tbi0 == 9 && (f.tbi1 == 8 || f.tbi1 == 9)) return kp != PSF_SR_FP16 ? 1 : f.tbi1 == 8 ? 2 : 4;
  if (f.tbi0 == 5 && f.tbi1 == 5 && f.tbj0 == 5) return 4;
  return kDefaultItemsPerCU;
}

// Persistent contraction workgroups for a launch of `items` work items of
// this family in precision kp: one per CU, two where the kernel runs two.
int64_t launch_wgs(const TilePlan& t, int64_t items, int kp) {
  return std::min<int64_t>(items, static_cast<int64_t>(kComputeUnits) * tile_wgs_per_cu(t, kp));
}
constexpr int kMaxDefaultItemsPerCU = 4;

Tuning tuning_for(const std::vector<Tuning>& table, const Family& f, int kp) {
  for (const Tuning& t : table)
    if (t.fam == f) return t;
  return {f, default_items_per_cu(f, kp), kFlushChunks};
}

// Group boundaries: sources ordered by family (stable), then cut into groups
// of one family, at most kMaxBatch sources and kRecordBudget record bytes.
struct Group {
  Family fam;
  std::vector<int> idx;
};

int group_capacity(const psf_obs* o) {
  const size_t rec = static_cast<size_t>(std::max<int64_t>(o->K, 1)) * (sizeof(BinRec) + sizeof(float2));
  return static_cast<int>(std::max<size_t>(1, std::min<size_t>(kMaxBatch, kRecordBudget / rec)));
}

std::vector<Group> make_groups(const psf_obs* o, int n_src, const psf_src* h) {
  std::vector<Family> fams;
  for (int s = 0; s < n_src; ++s) {
    const Family f = family_of(h[s]);
    if (std::find(fams.begin(), fams.end(), f) == fams.end()) fams.push_back(f);
  }
  const int cap = group_capacity(o);
  std::vector<Group> groups;
  for (const Family& f : fams) {
    Group g{f, {}};
    for (int s = 0; s < n_src; ++s) {
      if (!(family_of(h[s]) == f)) continue;
      g.idx.push_back(s);
      if (static_cast<int>(g.idx.size()) == cap) {
        groups.push_back(g);
        g.idx.clear();
      }
    }
    if (!g.idx.empty()) groups.push_back(g);
  }
  return groups;
}

struct GroupPlan {
  std::vector<PatchPlan> plans;
  int64_t items = 0;
  size_t partial_elems = 0;
};

GroupPlan plan_group(const psf_obs* o, const psf_src* h, const Group& g, int prec, int items_per_cu) {
  GroupPlan gp;
  double work = 0.0;
  for (int s : g.idx) work += patch_work(o, &h[s], prec);
  const double item_work = work / (static_cast<double>(kComputeUnits) * items_per_cu);
  for (int s : g.idx) {
    gp.plans.push_back(plan_patch_items(o, &h[s], prec, item_work));
    gp.items += tile_plan_items(gp.plans.back().tp);
    gp.partial_elems += align_up(gp.plans.back().partial_elems, 64);
  }
  return gp;
}

size_t records_bytes(const psf_obs* o) {
  return align_up(static_cast<size_t>(o->K) * sizeof(BinRec), 256) +
         align_up(static_cast<size_t>(o->K) * sizeof(float2), 256);
}

// Workspace: [records of up to group_capacity sources][partial slabs of the
// largest group, for the largest items-per-CU a tuning table may ask][the
// normalisation peaks of up to kMaxBatch sources].
size_t batch_workspace_for(const psf_obs* o, int n_src, const psf_src* h, int prec, int max_items_per_cu) {
  const std::vector<Group> groups = make_groups(o, n_src, h);
  size_t rec = 0, part = 0;
  for (const Group& g : groups) {
    rec = std::max(rec, g.idx.size() * records_bytes(o));
    part = std::max(part, plan_group(o, h, g, prec, max_items_per_cu).partial_elems * sizeof(float));
  }
  return align_up(rec, 256) + align_up(part, 256) + kMaxBatch * kPeakBytes;
}

int run_batched(const psf_obs* obs, int n_src, const psf_src* h, const psf_src* d, int prec, bool norm,
                const std::vector<Tuning>& table, float* P_all, void* ws, hipStream_t st, size_t peak_off) {
  const std::vector<Group> groups = make_groups(obs, n_src, h);
  const size_t rec = records_bytes(obs);
  size_t rec_area = 0;
  for (const Group& g : groups) rec_area = std::max(rec_area, g.idx.size() * rec);
  uint8_t* base = static_cast<uint8_t*>(ws);
  float* partial = reinterpret_cast<float*>(base + align_up(rec_area, 256));
  const ObsView ov = view(obs);
  for (const Group& g : groups) {
    const Tuning tu = tuning_for(table, g.fam, launch_prec(prec, obs->K, g.fam.sym != 0));
    const GroupPlan gp = plan_group(obs, h, g, prec, tu.items_per_cu);
    BatchArgs a;
    a.n_src = static_cast<int>(g.idx.size());
    a.flush_chunks = tu.flush;
    a.K = obs->K;
    a.n_items = gp.items;
    int64_t item0 = 0;
    size_t poff = 0;
    for (int q = 0; q < a.n_src; ++q) {
      const int s = g.idx[q];
      uint8_t* r = base + q * rec;
      BinRec* rec = reinterpret_cast<BinRec*>(r);
      float2* c = reinterpret_cast<float2*>(r + align_up(static_cast<size_t>(obs->K) * sizeof(BinRec), 256));
      const double* dir = reinterpret_cast<const double*>(d + s);
      if (obs->K > 0) {
        hipError_t e = launch_decorr_sources(ov, dir, 0, 1, rec, c, 0, st);
        if (e != hipSuccess) return hip_fail(e, "k_decorr launch");
      }
      double* peak = reinterpret_cast<double*>(base + peak_off + q * kPeakBytes);
      if (norm) {
        hipError_t e = launch_peak(c, obs->K, peak + 1, peak, st);
        if (e != hipSuccess) return hip_fail(e, "peak launch");
      }
      a.src[q] = src_plan(&h[s], gp.plans[q], rec, c, partial + poff, P_all + h[s].out_off, dir,
                          norm ? peak : nullptr);
      a.src[q].item0 = item0;
      item0 += tile_plan_items(gp.plans[q].tp);
      poff += align_up(gp.plans[q].partial_elems, 64);
    }
    const int64_t n_wg = launch_wgs(gp.plans[0].tp, gp.items, contraction_prec(prec, a));
    int rc = run_batch(prec, a, n_wg, st);
    if (rc != PSF_OK) return rc;
  }
  return PSF_OK;
}

int validate_batch(const psf_obs* obs, int32_t n_src, const psf_src* h_srcs, int prec) {
  int st;
  if ((st = validate_obs(obs)) != PSF_OK) return st;
  if ((st = validate_prec(prec)) != PSF_OK) return st;
  if (n_src < 1 || h_srcs == nullptr) return fail(PSF_EINVAL, "need n_src >= 1 sources");
  for (int s = 0; s < n_src; ++s)
    if ((st = validate_src(&h_srcs[s], s)) != PSF_OK) return st;
  return PSF_OK;
}

}  // namespace

// psf_autotune: the records of one source, partial slabs of one patch at
// the largest candidate, and one output patch.
size_t autotune_workspace(const psf_obs* o, int n_src, const psf_src* h, int prec) {
  size_t part = 0, pix = 0;
  for (int q = 0; q < n_src; ++q) {
    const double iw = patch_work(o, &h[q], prec) / (static_cast<double>(kComputeUnits) * kMaxItemsPerCU);
    part = std::max(part, plan_patch_items(o, &h[q], prec, iw).partial_elems);
    pix = std::max(pix, static_cast<size_t>(h[q].nl) * h[q].nm);
  }
  return records_bytes(o) + align_up(part * sizeof(float), 256) + align_up(pix * sizeof(float), 256);
}

size_t batched_workspace(const psf_obs* o, int n_src, const psf_src* h_srcs, int prec) {
  return std::max(batch_workspace_for(o, n_src, h_srcs, prec, kMaxItemsPerCU),
                  autotune_workspace(o, n_src, h_srcs, prec));
}

}  // namespace psf

using namespace psf;
extern "C" {

int psf_patch_batched(const psf_obs* obs, int32_t n_src, const psf_src* h_srcs, const psf_src* d_srcs, int prec,
                      const char* tuning_json, float* P_all, void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  int st;
  if ((st = validate_batch(obs, n_src, h_srcs, prec)) != PSF_OK) return st;
  const bool norm = prec_normalise(prec);
  prec = prec_base(prec);
  if (d_srcs == nullptr || P_all == nullptr) return fail(PSF_EINVAL, "d_srcs or P_all is NULL");
  std::vector<Tuning> table;
  if ((st = parse_tuning(tuning_json, &table)) != PSF_OK) return st;
  int mx = kMaxDefaultItemsPerCU;
  for (const Tuning& t : table) mx = std::max(mx, t.items_per_cu);
  const size_t need = batch_workspace_for(obs, n_src, h_srcs, prec, mx);
  if (ws == nullptr || ws_bytes < need)
    return fail(PSF_EWORKSPACE, "psf_patch_batched needs %zu workspace bytes, got %zu", need, ws_bytes);
  if ((st = check_device()) != PSF_OK) return st;
  return run_batched(obs, n_src, h_srcs, d_srcs, prec, norm, table, P_all, ws, static_cast<hipStream_t>(stream),
                     need - kMaxBatch * kPeakBytes);
}

int psf_autotune(const psf_obs* obs, int32_t n_src, const psf_src* h_srcs, int prec, void* ws, size_t ws_bytes,
                 char* json_out, size_t json_cap, void* stream) {
  clear_error();
  int st;
  if ((st = validate_batch(obs, n_src, h_srcs, prec)) != PSF_OK) return st;
  prec = prec_base(prec);  // normalisation does not change the launch shapes
  if (json_out == nullptr || json_cap < 64) return fail(PSF_EINVAL, "json_out missing or too small");
  if ((st = check_device()) != PSF_OK) return st;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  // One representative source per family (its first), contracted from its
  // own records with every candidate launch shape; fastest wins.
  std::vector<Family> fams;
  std::vector<int> rep;
  for (int q = 0; q < n_src; ++q) {
    const Family f = family_of(h_srcs[q]);
    if (std::find(fams.begin(), fams.end(), f) == fams.end()) {
      fams.push_back(f);
      rep.push_back(q);
    }
  }
  size_t part = 0;
  for (int q : rep)
    for (int ipc : kItemsCandidates) {
      const double iw = patch_work(obs, &h_srcs[q], prec) / (static_cast<double>(kComputeUnits) * ipc);
      part = std::max(part, plan_patch_items(obs, &h_srcs[q], prec, iw).partial_elems);
    }
  const size_t need = autotune_workspace(obs, n_src, h_srcs, prec);
  if (ws == nullptr || ws_bytes < need)
    return fail(PSF_EWORKSPACE, "psf_autotune needs %zu workspace bytes, got %zu", need, ws_bytes);
  uint8_t* w = static_cast<uint8_t*>(ws);
  BinRec* rec = reinterpret_cast<BinRec*>(w);
  float2* c = reinterpret_cast<float2*>(w + align_up(static_cast<size_t>(obs->K) * sizeof(BinRec), 256));
  float* partial = reinterpret_cast<float*>(w + records_bytes(obs));
  float* P = reinterpret_cast<float*>(w + records_bytes(obs) + align_up(part * sizeof(float), 256));

  hipEvent_t e0, e1;
  hipError_t e;
  if ((e = hipEventCreate(&e0)) != hipSuccess) return hip_fail(e, "hipEventCreate");
  if ((e = hipEventCreate(&e1)) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_fail(e, "hipEventCreate");
  }
  std::string out = "{\"prec\": " + std::to_string(prec) + ", \"families\": [";
  int rc = PSF_OK;
  for (size_t f = 0; f < fams.size() && rc == PSF_OK; ++f) {
    const psf_src& src = h_srcs[rep[f]];
    if (obs->K > 0 &&
        (e = launch_decorr(view(obs), src.l0, src.m0, src.dl, src.dm, nullptr, nullptr, rec, c, nullptr, s)) !=
            hipSuccess) {
      rc = hip_fail(e, "k_decorr launch");
      break;
    }
    double best_ms = 1e30;
    int best_ipc = kDefaultItemsPerCU, best_flush = kFlushChunks;
    for (int ipc : kItemsCandidates) {
      for (int fl : kFlushCandidates) {
        const double iw = patch_work(obs, &src, prec) / (static_cast<double>(kComputeUnits) * ipc);
        const PatchPlan plan = plan_patch_items(obs, &src, prec, iw);
        BatchArgs a;
        a.n_src = 1;
        a.flush_chunks = fl;
        a.K = obs->K;
        a.src[0] = src_plan(&src, plan, rec, c, partial, P, nullptr);
        a.n_items = tile_plan_items(plan.tp);
        const int64_t n_wg = launch_wgs(plan.tp, a.n_items, contraction_prec(prec, a));
        constexpr int kReps = 3;
        const int kp = contraction_prec(prec, a);
        if ((e = launch_patch(kp, a, n_wg, s)) != hipSuccess) {  // warm-up
          rc = hip_fail(e, "k_patch launch");
          break;
        }
        if ((e = hipEventRecord(e0, s)) != hipSuccess) {
          rc = hip_fail(e, "hipEventRecord");
          break;
        }
        for (int r = 0; r < kReps && e == hipSuccess; ++r) e = launch_patch(kp, a, n_wg, s);
        if (e != hipSuccess) {
          rc = hip_fail(e, "k_patch launch");
          break;
        }
        float ms = 0.f;
        if ((e = hipEventRecord(e1, s)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess ||
            (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) {
          rc = hip_fail(e, "timing events");
          break;
        }
        ms /= kReps;
        if (ms < best_ms) {
          best_ms = ms;
          best_ipc = ipc;
          best_flush = fl;
        }
      }
      if (rc != PSF_OK) break;
    }
    if (rc != PSF_OK) break;
    char buf[256];
    std::snprintf(buf, sizeof buf,
                  "%s{\"tbi0\": %d, \"tbi1\": %d, \"tbj0\": %d, \"tbj1\": %d, \"sym\": %d, "
                  "\"items_per_cu\": %d, \"flush\": %d, \"ms\": %.4f, \"nl\": %d, \"nm\": %d}",
                  f ? ", " : "", fams[f].tbi0, fams[f].tbi1, fams[f].tbj0, fams[f].tbj1, fams[f].sym, best_ipc,
                  best_flush, best_ms, src.nl, src.nm);
    out += buf;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != PSF_OK) return rc;
  out += "]}";
  if (out.size() + 1 > json_cap) return fail(PSF_EINVAL, "json_out needs %zu bytes", out.size() + 1);
  std::memcpy(json_out, out.c_str(), out.size() + 1);
  return PSF_OK;
}

}  // extern "C"
