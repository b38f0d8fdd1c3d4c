// extern "C" entry points of libttnn.so.  Each wraps its body so that no C++
// exception crosses the ABI; statuses and messages follow include/ttnn.h.
#include <algorithm>
#include <cstring>
#include <map>
#include <vector>
#include <string>

#include "engine.hpp"
#include "kernels.hpp"
#include "kr.hpp"
#include "order.hpp"

struct ttnn_plan_s {
  std::unique_ptr<ttnn::Plan> p;
};

namespace ttnn {

thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }
const char* last_error() { return g_last_error.c_str(); }

}  // namespace ttnn

namespace {

using ttnn::Error;
using ttnn::Plan;

hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

template <typename F>
ttnn_status guard(Plan* P, F&& body) {
  try {
    if (P && P->sticky != TTNN_OK) {
      ttnn::set_error("plan has a sticky error from an earlier call; call ttnn_reset");
      return P->sticky;
    }
    return body();
  } catch (const Error& e) {
    ttnn::set_error(e.msg);
    if (P && e.status == TTNN_E_HIP) P->sticky = TTNN_E_HIP;
    return e.status;
  } catch (const std::exception& e) {
    ttnn::set_error(e.what());
    return TTNN_E_INVALID;
  }
}

Plan* get(ttnn_plan_t h) { return h ? h->p.get() : nullptr; }

int level_id(const Plan& P, int32_t node) {
  if (node < 0 || node >= static_cast<int32_t>(P.level_of_caller.size()))
    throw Error{TTNN_E_RANGE, "node id out of range"};
  return P.level_of_caller[node];
}

void check_box(const Plan& P, const int64_t* off, const int64_t* ext, bool* empty) {
  if (!off || !ext) throw Error{TTNN_E_INVALID, "offset/extent is NULL"};
  *empty = false;
  for (int mu = 0; mu < P.d; ++mu) {
    if (off[mu] < 0 || ext[mu] < 0 || off[mu] + ext[mu] > P.dims[mu])
      throw Error{TTNN_E_RANGE, "update box outside the tensor in mode " + std::to_string(mu)};
    if (ext[mu] == 0) *empty = true;
  }
}

// Validated strides of a block, or nullptr when the block is packed (strides equal to
// the packed column-major ones on every mode of extent > 1, or strides absent).
const int64_t* block_strides(const Plan& P, const int64_t* ext, const int64_t* strides) {
  if (!strides) return nullptr;
  bool packed = true;
  int64_t pk = 1;
  for (int mu = 0; mu < P.d; ++mu) {
    if (ext[mu] > 1) {
      if (strides[mu] < 1) throw Error{TTNN_E_INVALID, "strides must be >= 1 on modes of extent > 1"};
      if (strides[mu] != pk) packed = false;
    }
    pk *= ext[mu];
  }
  return packed ? nullptr : strides;
}

// A large strided block packed into a stream-ordered pool block (returned to the pool in
// stream order when the holder goes, after the update that reads it is enqueued).
struct Packed {
  void* p = nullptr;
  hipStream_t s = nullptr;
  Packed() = default;
  Packed(const Packed&) = delete;
  Packed(Packed&& o) noexcept : p(o.p), s(o.s) { o.p = nullptr; }
  ~Packed() {
    if (p) ttnn::pool_free(p, s);
  }
};

bool pack_large(const Plan& P, const void* block, const int64_t* ext, const int64_t* strides, hipStream_t st,
                Packed& out) {
  if (!strides) return false;
  int64_t entries = 1;
  for (int mu = 0; mu < P.d; ++mu) entries *= ext[mu];
  if (entries < ttnn::kPackMinEntries) return false;
  out.s = st;
  out.p = ttnn::pool_alloc(static_cast<size_t>(entries) * ttnn::dtype_size(P.dtype), st);
  ttnn::launch_pack_box(block, P.dtype, P.d, ext, strides, out.p, st);
  return true;
}

void dense_updates(const Plan& P) {
  if (P.variant == TTNN_KR)
    throw Error{TTNN_E_STATE, "a Khatri-Rao plan takes TTN-format updates only (ttnn_sketch_update_ttn)"};
}

// Level-order ranks of a TTN from the caller's array (root entry ignored).
std::vector<int64_t> ttn_ranks(const Plan& P, const int32_t* ranks) {
  if (!ranks) throw Error{TTNN_E_INVALID, "ranks is NULL"};
  std::vector<int64_t> s(P.nodes.size(), 1);
  for (size_t c = 0; c < P.level_of_caller.size(); ++c) {
    const int v = P.level_of_caller[c];
    if (v > 0) s[v] = ranks[c];
  }
  return s;
}

std::vector<const double*> ttn_cores(const Plan& P, const double* const* cores) {
  if (!cores) throw Error{TTNN_E_INVALID, "cores is NULL"};
  std::vector<const double*> by_level(P.nodes.size());
  for (size_t c = 0; c < P.level_of_caller.size(); ++c) {
    if (!cores[c]) throw Error{TTNN_E_INVALID, "core pointer is NULL"};
    by_level[P.level_of_caller[c]] = cores[c];
  }
  return by_level;
}

// Scratch for one call: the caller's (checked), else from the pool for the call.
struct CallWork {
  void* p = nullptr;
  bool owned = false;
  hipStream_t st = nullptr;
  CallWork(void* d_work, size_t have, size_t need, hipStream_t s) : st(s) {
    if (d_work) {
      if (have < need)
        throw Error{TTNN_E_INVALID, "work buffer of " + std::to_string(have) + " bytes; the call needs " +
                                        std::to_string(need)};
      if (reinterpret_cast<uintptr_t>(d_work) % 256 != 0) throw Error{TTNN_E_INVALID, "work buffer not 256-byte aligned"};
      p = d_work;
    } else {
      p = ttnn::pool_alloc(need, s);
      owned = true;
    }
  }
  ~CallWork() {
    if (owned) ttnn::pool_free(p, st);
  }
};

}  // namespace

extern "C" {

ttnn_status ttnn_plan_create(const ttnn_problem* problem, void* stream, ttnn_plan_t* out) {
  return guard(nullptr, [&]() -> ttnn_status {
    if (!out) throw Error{TTNN_E_INVALID, "out is NULL"};
    *out = nullptr;
    auto P = ttnn::build_plan(problem, as_stream(stream));
    auto* h = new ttnn_plan_s;
    h->p = std::move(P);
    *out = h;
    return TTNN_OK;
  });
}

size_t ttnn_workspace_bytes(const ttnn_problem* problem) {
  try {
    return ttnn::build_plan(problem, nullptr, /*dry=*/true)->footprint;
  } catch (const Error& e) {
    ttnn::set_error(e.msg);
  } catch (const std::exception& e) {
    ttnn::set_error(e.what());
  }
  return 0;
}

ttnn_status ttnn_plan(const ttnn_problem* problem, void* d_ws, size_t ws_bytes, void* stream, ttnn_plan_t* out) {
  return guard(nullptr, [&]() -> ttnn_status {
    if (!out) throw Error{TTNN_E_INVALID, "out is NULL"};
    *out = nullptr;
    if (!d_ws) throw Error{TTNN_E_INVALID, "workspace is NULL"};
    if (reinterpret_cast<uintptr_t>(d_ws) % 256 != 0) throw Error{TTNN_E_INVALID, "workspace not 256-byte aligned"};
    auto P = ttnn::build_plan(problem, as_stream(stream), false, d_ws, ws_bytes);
    auto* h = new ttnn_plan_s;
    h->p = std::move(P);
    *out = h;
    return TTNN_OK;
  });
}

ttnn_status ttnn_destroy(ttnn_plan_t plan) {
  if (!plan) return TTNN_OK;
  (void)hipDeviceSynchronize();
  delete plan;
  return TTNN_OK;
}

ttnn_status ttnn_destroy_async(ttnn_plan_t plan, void* stream) {
  if (!plan) return TTNN_OK;
  plan->p->free_stream = as_stream(stream);
  delete plan;
  return TTNN_OK;
}

size_t ttnn_footprint_bytes(ttnn_plan_t plan) { return plan ? plan->p->footprint : 0; }

ttnn_status ttnn_sketch_update(ttnn_plan_t plan, const void* d_block, const int64_t* offset, const int64_t* extent,
                               const int64_t* strides, double alpha, void* stream) {
  Plan* P = get(plan);
  return guard(P, [&]() -> ttnn_status {
    if (!P) throw Error{TTNN_E_INVALID, "plan is NULL"};
    dense_updates(*P);
    bool empty = false;
    check_box(*P, offset, extent, &empty);
    if (empty) return TTNN_OK;
    if (!d_block) throw Error{TTNN_E_INVALID, "block is NULL"};
    const int64_t* st = block_strides(*P, extent, strides);
    Packed pk;
    if (pack_large(*P, d_block, extent, st, as_stream(stream), pk))
      ttnn::update_box(*P, pk.p, offset, extent, nullptr, alpha, as_stream(stream));
    else
      ttnn::update_box(*P, d_block, offset, extent, st, alpha, as_stream(stream));
    TTNN_HIP(hipGetLastError());
    return TTNN_OK;
  });
}

ttnn_status ttnn_sketch_update_rank1(ttnn_plan_t plan, const double* const* d_factors, double alpha, void* stream) {
  Plan* P = get(plan);
  return guard(P, [&]() -> ttnn_status {
    if (!P || !d_factors) throw Error{TTNN_E_INVALID, "plan or factors is NULL"};
    dense_updates(*P);
    for (int mu = 0; mu < P->d; ++mu)
      if (!d_factors[mu]) throw Error{TTNN_E_INVALID, "factor pointer is NULL"};
    ttnn::update_rank1(*P, 1, d_factors, &alpha, as_stream(stream));
    TTNN_HIP(hipGetLastError());
    return TTNN_OK;
  });
}

ttnn_status ttnn_sketch_update_rank1_batched(ttnn_plan_t plan, int32_t nterms, const double* const* d_factors,
                                             const double* alphas, void* stream) {
  Plan* P = get(plan);
  return guard(P, [&]() -> ttnn_status {
    if (!P || nterms < 0 || (nterms > 0 && (!d_factors || !alphas)))
      throw Error{TTNN_E_INVALID, "plan, factors or alphas is NULL, or nterms < 0"};
    dense_updates(*P);
    for (int64_t e = 0; e < static_cast<int64_t>(nterms) * P->d; ++e)
      if (!d_factors[e]) throw Error{TTNN_E_INVALID, "factor pointer is NULL"};
    ttnn::update_rank1(*P, nterms, d_factors, alphas, as_stream(stream));
    TTNN_HIP(hipGetLastError());
    return TTNN_OK;
  });
}

ttnn_status ttnn_sketch_update_batched(int32_t n, const ttnn_update_desc* descs, void* stream) {
  return guard(nullptr, [&]() -> ttnn_status {
    if (n < 0 || (n > 0 && !descs)) throw Error{TTNN_E_INVALID, "bad descriptor array"};
    // validate everything before enqueueing anything
    for (int32_t i = 0; i < n; ++i) {
      Plan* P = get(descs[i].plan);
      if (!P) throw Error{TTNN_E_INVALID, "descriptor " + std::to_string(i) + " has no plan"};
      if (P->sticky != TTNN_OK) throw Error{P->sticky, "descriptor plan has a sticky error"};
      dense_updates(*P);
      bool empty = false;
      check_box(*P, descs[i].offset, descs[i].extent, &empty);
      if (!empty && !descs[i].d_block) throw Error{TTNN_E_INVALID, "descriptor block is NULL"};
      if (!empty && descs[i].strides[0] != 0) block_strides(*P, descs[i].extent, descs[i].strides);
    }
    std::vector<int32_t> pending;
    for (int32_t i = 0; i < n; ++i) {
      bool empty = false;
      check_box(*get(descs[i].plan), descs[i].offset, descs[i].extent, &empty);
      if (!empty) pending.push_back(i);
    }
    const hipStream_t st = as_stream(stream);
    try {
      // Rounds: each round takes the earliest pending update of every plan (so a plan's
      // updates keep their order); the box updates of a round whose plans share a tree
      // shape, variant and dtype run as one launch per step.
      while (!pending.empty()) {
        std::vector<int32_t> round, rest;
        std::vector<Plan*> seen;
        for (int32_t i : pending) {
          Plan* P = get(descs[i].plan);
          if (std::find(seen.begin(), seen.end(), P) != seen.end()) {
            rest.push_back(i);
            continue;
          }
          seen.push_back(P);
          round.push_back(i);
        }
        std::map<std::string, std::vector<int32_t>> buckets;
        // large strided blocks are packed first (held until the round is enqueued)
        std::map<int32_t, Packed> packed;
        for (int32_t i : round) {
          const ttnn_update_desc& u = descs[i];
          const int64_t* s = u.strides[0] != 0 ? block_strides(*get(u.plan), u.extent, u.strides) : nullptr;
          Packed pk;
          if (pack_large(*get(u.plan), u.d_block, u.extent, s, st, pk)) packed.emplace(i, std::move(pk));
        }
        auto block_of = [&](int32_t i) -> const void* {
          auto it = packed.find(i);
          return it != packed.end() ? it->second.p : descs[i].d_block;
        };
        auto strides_of = [&](int32_t i) -> const int64_t* {
          const ttnn_update_desc& u = descs[i];
          if (packed.count(i)) return nullptr;
          return u.strides[0] != 0 ? block_strides(*get(u.plan), u.extent, u.strides) : nullptr;
        };
        for (int32_t i : round) {
          Plan* P = get(descs[i].plan);
          if (ttnn::whole_tensor(*P, descs[i].offset, descs[i].extent) && !strides_of(i))
            ttnn::update_box(*P, block_of(i), descs[i].offset, descs[i].extent, nullptr, descs[i].alpha, st);
          else
            buckets[ttnn::batch_key(*P)].push_back(i);
        }
        for (auto& kv : buckets) {
          std::vector<std::vector<ttnn::BoxOp>> recs(kv.second.size());
          std::vector<const std::vector<ttnn::BoxOp>*> items;
          std::vector<Plan*> plans;
          for (size_t b = 0; b < kv.second.size(); ++b) {
            const int32_t i = kv.second[b];
            Plan* P = get(descs[i].plan);
            P->epilogue_valid = false;
            ttnn::record_box(*P, block_of(i), descs[i].offset, descs[i].extent, strides_of(i), descs[i].alpha,
                             recs[b]);
            items.push_back(&recs[b]);
            plans.push_back(P);
          }
          ttnn::run_box_ops_batched(plans, items, st);
        }
        TTNN_HIP(hipGetLastError());
        pending.swap(rest);
      }
    } catch (const Error& e) {
      if (e.status == TTNN_E_HIP)
        for (int32_t i = 0; i < n; ++i) get(descs[i].plan)->sticky = TTNN_E_HIP;
      throw;
    }
    return TTNN_OK;
  });
}

ttnn_status ttnn_footprint_estimate(const ttnn_problem* problem, size_t* bytes) {
  return guard(nullptr, [&]() -> ttnn_status {
    if (!bytes) throw Error{TTNN_E_INVALID, "bytes is NULL"};
    *bytes = 0;
    auto P = ttnn::build_plan(problem, nullptr, /*dry=*/true);
    *bytes = P->footprint;
    return TTNN_OK;
  });
}

ttnn_status ttnn_order_cost(const ttnn_problem* problem, int32_t objective, double* cost) {
  return guard(nullptr, [&]() -> ttnn_status {
    if (!cost) throw Error{TTNN_E_INVALID, "cost is NULL"};
    if (objective != TTNN_COST_FLOPS && objective != TTNN_COST_MAPS) throw Error{TTNN_E_INVALID, "bad objective"};
    auto P = ttnn::build_plan(problem, nullptr, /*dry=*/true);
    if (P->variant != TTNN_STTNN) throw Error{TTNN_E_INVALID, "visiting orders concern STTNN plans"};
    *cost = ttnn::order_cost(*P, objective);
    return TTNN_OK;
  });
}

ttnn_status ttnn_order_search(const ttnn_problem* problem, int32_t objective, int32_t* visit, double* cost) {
  return guard(nullptr, [&]() -> ttnn_status {
    if (!visit || !cost) throw Error{TTNN_E_INVALID, "NULL argument"};
    if (objective != TTNN_COST_FLOPS && objective != TTNN_COST_MAPS) throw Error{TTNN_E_INVALID, "bad objective"};
    auto P = ttnn::build_plan(problem, nullptr, /*dry=*/true);
    if (P->variant != TTNN_STTNN) throw Error{TTNN_E_INVALID, "visiting orders concern STTNN plans"};
    const std::vector<int> place = ttnn::order_search(*P, objective, cost);
    for (size_t i = 0; i < place.size(); ++i) visit[i] = place[i];
    return TTNN_OK;
  });
}

ttnn_status ttnn_update_ttn_work_bytes(ttnn_plan_t plan, const int32_t* ranks, size_t* bytes) {
  Plan* P = get(plan);
  return guard(nullptr, [&]() -> ttnn_status {
    if (!P || !bytes) throw Error{TTNN_E_INVALID, "NULL argument"};
    if (P->variant != TTNN_KR) throw Error{TTNN_E_STATE, "TTN-format updates need a Khatri-Rao plan"};
    *bytes = ttnn::kr_update_work_bytes(*P, ttn_ranks(*P, ranks));
    return TTNN_OK;
  });
}

ttnn_status ttnn_sketch_update_ttn(ttnn_plan_t plan, const double* const* d_cores, const int32_t* ranks, double alpha,
                                   void* d_work, size_t work_bytes, void* stream) {
  Plan* P = get(plan);
  return guard(P, [&]() -> ttnn_status {
    if (!P) throw Error{TTNN_E_INVALID, "plan is NULL"};
    if (P->variant != TTNN_KR) throw Error{TTNN_E_STATE, "TTN-format updates need a Khatri-Rao plan"};
    const auto s = ttn_ranks(*P, ranks);
    const auto cores = ttn_cores(*P, d_cores);
    const size_t need = ttnn::kr_update_work_bytes(*P, s);
    const hipStream_t st = as_stream(stream);
    CallWork w(d_work, work_bytes, need, st);
    ttnn::update_ttn(*P, cores.data(), s, alpha, w.p, st);
    TTNN_HIP(hipGetLastError());
    return TTNN_OK;
  });
}

ttnn_status ttnn_ttn_dot_work_bytes(ttnn_plan_t plan, const int32_t* ranks_a, const int32_t* ranks_b, size_t* bytes) {
  Plan* P = get(plan);
  return guard(nullptr, [&]() -> ttnn_status {
    if (!P || !bytes) throw Error{TTNN_E_INVALID, "NULL argument"};
    if (P->nodes.size() != static_cast<size_t>(P->n_real))
      throw Error{TTNN_E_TREE, "TTN inner products take trees without free modes"};
    *bytes = ttnn::ttn_dot_work_bytes(*P, ttn_ranks(*P, ranks_a), ttn_ranks(*P, ranks_b));
    return TTNN_OK;
  });
}

ttnn_status ttnn_ttn_dot(ttnn_plan_t plan, const double* const* d_a, const int32_t* ranks_a, const double* const* d_b,
                         const int32_t* ranks_b, double* d_out, void* d_work, size_t work_bytes, void* stream) {
  Plan* P = get(plan);
  return guard(P, [&]() -> ttnn_status {
    if (!P || !d_out) throw Error{TTNN_E_INVALID, "NULL argument"};
    if (P->nodes.size() != static_cast<size_t>(P->n_real))
      throw Error{TTNN_E_TREE, "TTN inner products take trees without free modes"};
    const auto sa = ttn_ranks(*P, ranks_a), sb = ttn_ranks(*P, ranks_b);
    const auto a = ttn_cores(*P, d_a), b = ttn_cores(*P, d_b);
    const size_t need = ttnn::ttn_dot_work_bytes(*P, sa, sb);
    const hipStream_t st = as_stream(stream);
    CallWork w(d_work, work_bytes, need, st);
    ttnn::ttn_dot(*P, a.data(), sa, b.data(), sb, d_out, w.p, st);
    TTNN_HIP(hipGetLastError());
    return TTNN_OK;
  });
}

ttnn_status ttnn_read_factor(ttnn_plan_t plan, int32_t mode, int32_t kind, double* d_out, void* stream) {
  Plan* P = get(plan);
  return guard(P, [&]() -> ttnn_status {
    if (!P || !d_out) throw Error{TTNN_E_INVALID, "NULL argument"};
    if (P->variant != TTNN_KR) throw Error{TTNN_E_STATE, "only Khatri-Rao plans have per-mode factors"};
    if (mode < 0 || mode >= P->d) throw Error{TTNN_E_RANGE, "mode out of range"};
    if (kind != 0 && kind != 1) throw Error{TTNN_E_INVALID, "bad factor kind"};
    const int cols = kind == 0 ? P->nodes[1].r : P->nodes[1].k;
    ttnn::launch_copy_f64(d_out, kind == 0 ? P->kr_x[mode] : P->kr_y[mode], P->dims[mode] * cols, as_stream(stream));
    TTNN_HIP(hipGetLastError());
    return TTNN_OK;
  });
}

ttnn_status ttnn_core_shape(ttnn_plan_t plan, int32_t node, int32_t* ndim, int64_t* shape) {
  Plan* P = get(plan);
  return guard(nullptr, [&]() -> ttnn_status {
    if (!P || !ndim || !shape) throw Error{TTNN_E_INVALID, "NULL argument"};
    const auto s = ttnn::core_shape(*P, level_id(*P, node));
    *ndim = static_cast<int32_t>(s.size());
    for (size_t i = 0; i < s.size(); ++i) shape[i] = s[i];
    return TTNN_OK;
  });
}

ttnn_status ttnn_assemble(ttnn_plan_t plan, double* const* d_cores, void* stream) {
  Plan* P = get(plan);
  return guard(P, [&]() -> ttnn_status {
    if (!P || !d_cores) throw Error{TTNN_E_INVALID, "NULL argument"};
    std::vector<double*> by_level(P->nodes.size());
    for (size_t c = 0; c < P->level_of_caller.size(); ++c) {
      if (!d_cores[c]) throw Error{TTNN_E_INVALID, "core pointer is NULL"};
      by_level[P->level_of_caller[c]] = d_cores[c];
    }
    const ttnn_status s = ttnn::run_assemble(*P, by_level.data(), as_stream(stream));
    TTNN_HIP(hipGetLastError());
    if (s != TTNN_OK) ttnn::set_error("non-finite sketch, or a node whose Omega has numerical rank 0");
    return s;
  });
}

ttnn_status ttnn_assemble_async(ttnn_plan_t plan, double* const* d_cores, void* stream) {
  Plan* P = get(plan);
  return guard(P, [&]() -> ttnn_status {
    if (!P || !d_cores) throw Error{TTNN_E_INVALID, "NULL argument"};
    std::vector<double*> by_level(P->nodes.size());
    for (size_t c = 0; c < P->level_of_caller.size(); ++c) {
      if (!d_cores[c]) throw Error{TTNN_E_INVALID, "core pointer is NULL"};
      by_level[P->level_of_caller[c]] = d_cores[c];
    }
    ttnn::enqueue_assemble(*P, by_level.data(), as_stream(stream));
    TTNN_HIP(hipGetLastError());
    return TTNN_OK;
  });
}

ttnn_status ttnn_assemble_status(ttnn_plan_t plan, void* stream) {
  Plan* P = get(plan);
  return guard(P, [&]() -> ttnn_status {
    if (!P) throw Error{TTNN_E_INVALID, "NULL argument"};
    const ttnn_status s = ttnn::assemble_status(*P, as_stream(stream));
    if (s != TTNN_OK) ttnn::set_error("an assembly since the last status query met a non-finite sketch, or a node "
                                      "whose Omega has numerical rank 0");
    return s;
  });
}

ttnn_status ttnn_assemble_status_async(ttnn_plan_t plan, int32_t* h_status, void* stream) {
  Plan* P = get(plan);
  return guard(P, [&]() -> ttnn_status {
    if (!P || !h_status) throw Error{TTNN_E_INVALID, "NULL argument"};
    ttnn::assemble_status_async(*P, h_status, as_stream(stream));
    TTNN_HIP(hipGetLastError());
    return TTNN_OK;
  });
}

ttnn_status ttnn_reconstruct(ttnn_plan_t plan, const double* const* d_cores, void* d_out, int32_t out_dtype,
                             void* stream) {
  Plan* P = get(plan);
  return guard(P, [&]() -> ttnn_status {
    if (!P || !d_cores || !d_out) throw Error{TTNN_E_INVALID, "NULL argument"};
    if (out_dtype != TTNN_F64 && out_dtype != TTNN_F32) throw Error{TTNN_E_INVALID, "out_dtype must be F64 or F32"};
    if (!P->recon_ok) throw Error{TTNN_E_STATE, "this Khatri-Rao plan sized no dense reconstruction (tensor too large)"};
    std::vector<const double*> by_level(P->nodes.size());
    for (size_t c = 0; c < P->level_of_caller.size(); ++c) {
      if (!d_cores[c]) throw Error{TTNN_E_INVALID, "core pointer is NULL"};
      by_level[P->level_of_caller[c]] = d_cores[c];
    }
    ttnn::run_reconstruct(*P, by_level.data(), d_out, out_dtype, as_stream(stream));
    TTNN_HIP(hipGetLastError());
    return TTNN_OK;
  });
}

ttnn_status ttnn_diff_norms(const void* d_a, int32_t a_dtype, const double* d_b, int64_t n, double* h_out,
                            void* stream) {
  return guard(nullptr, [&]() -> ttnn_status {
    if (!d_a || !d_b || !h_out || n < 0) throw Error{TTNN_E_INVALID, "bad argument"};
    if (a_dtype != TTNN_F64 && a_dtype != TTNN_F32 && a_dtype != TTNN_BF16) throw Error{TTNN_E_INVALID, "bad dtype"};
    hipStream_t st = as_stream(stream);
    // partial sums from the library's per-device pool, stream ordered (no device-wide
    // allocation or free per call)
    struct Block {                             // returned to the pool in stream order, also on errors
      void* p;
      hipStream_t s;
      ~Block() { ttnn::pool_free(p, s); }
    } blk{ttnn::pool_alloc(sizeof(double) * (2 * ttnn::kNormBlocks + 2), st), st};
    double* d_part = static_cast<double*>(blk.p);
    ttnn::launch_diff_norms(d_a, a_dtype, d_b, n, d_part, d_part + 2 * ttnn::kNormBlocks, st);
    TTNN_HIP(hipMemcpyAsync(h_out, d_part + 2 * ttnn::kNormBlocks, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    TTNN_HIP(hipStreamSynchronize(st));
    return TTNN_OK;
  });
}

ttnn_status ttnn_diff_norms_noalloc(const void* d_a, int32_t a_dtype, const double* d_b, int64_t n, double* d_out,
                                    void* stream) {
  return guard(nullptr, [&]() -> ttnn_status {
    if (!d_a || !d_b || !d_out || n < 0) throw Error{TTNN_E_INVALID, "bad argument"};
    if (a_dtype != TTNN_F64 && a_dtype != TTNN_F32 && a_dtype != TTNN_BF16) throw Error{TTNN_E_INVALID, "bad dtype"};
    ttnn::launch_diff_norms_static(d_a, a_dtype, d_b, n, d_out, as_stream(stream));
    TTNN_HIP(hipGetLastError());
    return TTNN_OK;
  });
}

ttnn_status ttnn_sketch_shape(ttnn_plan_t plan, int32_t node, int32_t kind, int64_t* rows, int64_t* cols) {
  Plan* P = get(plan);
  return guard(nullptr, [&]() -> ttnn_status {
    if (!P || !rows || !cols) throw Error{TTNN_E_INVALID, "NULL argument"};
    const int v = level_id(*P, node);
    const ttnn::Node& t = P->nodes[v];
    if (v == 0) {
      if (kind != TTNN_SK_PSI) throw Error{TTNN_E_RANGE, "the root only has a Psi sketch"};
      *rows = P->psi_root_len;
      *cols = 1;
      return TTNN_OK;
    }
    if (kind == TTNN_SK_R) { *rows = t.n; *cols = t.r; }
    else if (kind == TTNN_SK_OMEGA) { *rows = t.k; *cols = t.r; }
    else if (kind == TTNN_SK_PSI) {
      int64_t kk = 1;
      for (int c : t.children) kk *= P->nodes[c].k;
      *rows = t.leaf() ? t.n : kk;
      *cols = t.r;
    } else throw Error{TTNN_E_INVALID, "bad sketch kind"};
    return TTNN_OK;
  });
}

ttnn_status ttnn_read_sketch(ttnn_plan_t plan, int32_t node, int32_t kind, double* d_out, void* stream) {
  Plan* P = get(plan);
  return guard(P, [&]() -> ttnn_status {
    if (!P || !d_out) throw Error{TTNN_E_INVALID, "NULL argument"};
    int64_t rows = 0, cols = 0;
    const ttnn_status s = ttnn_sketch_shape(plan, node, kind, &rows, &cols);
    if (s != TTNN_OK) return s;
    const int v = level_id(*P, node);
    hipStream_t st = as_stream(stream);
    const ttnn::Node& t = P->nodes[v];
    const double* src = nullptr;
    if (v == 0) src = P->psi_root;
    else if (kind == TTNN_SK_R || (kind == TTNN_SK_PSI && t.leaf())) {
      if (!t.R) throw Error{TTNN_E_STATE, "a Khatri-Rao plan keeps no R_t of internal nodes"};
      src = t.R;
    }
    else {
      if (!P->epilogue_valid) ttnn::run_epilogue(*P, st);
      src = kind == TTNN_SK_OMEGA ? t.Om : t.Psi;
    }
    ttnn::launch_copy_f64(d_out, src, rows * cols, st);
    TTNN_HIP(hipGetLastError());
    return TTNN_OK;
  });
}

ttnn_status ttnn_drm_shape(ttnn_plan_t plan, int32_t node, int32_t kind, int64_t* rows, int64_t* cols) {
  Plan* P = get(plan);
  return guard(nullptr, [&]() -> ttnn_status {
    if (!P || !rows || !cols) throw Error{TTNN_E_INVALID, "NULL argument"};
    const int v = level_id(*P, node);
    if (v == 0) throw Error{TTNN_E_RANGE, "the root has no DRMs"};
    const ttnn::Node& t = P->nodes[v];
    if (kind == 0) { *rows = t.m; *cols = t.r; }
    else if (kind == 1) { *rows = t.n; *cols = t.k; }
    else throw Error{TTNN_E_INVALID, "bad DRM kind"};
    return TTNN_OK;
  });
}

ttnn_status ttnn_read_drm(ttnn_plan_t plan, int32_t node, int32_t kind, int32_t dtype, void* d_out, void* stream) {
  Plan* P = get(plan);
  return guard(P, [&]() -> ttnn_status {
    if (!P || !d_out) throw Error{TTNN_E_INVALID, "NULL argument"};
    int64_t rows = 0, cols = 0;
    const ttnn_status s = ttnn_drm_shape(plan, node, kind, &rows, &cols);
    if (s != TTNN_OK) return s;
    const ttnn::Node& t = P->nodes[level_id(*P, node)];
    if (P->variant == TTNN_KR) throw Error{TTNN_E_STATE, "a Khatri-Rao plan forms no dense maps (ttnn_read_factor)"};
    const void* src;
    if (dtype == TTNN_F64) src = kind == 0 ? t.X64 : t.Y64;
    else if (dtype == P->dtype) src = kind == 0 ? t.Xc : t.Yc;
    else throw Error{TTNN_E_INVALID, "the plan stores no DRM copy of that dtype"};
    TTNN_HIP(hipMemcpyAsync(d_out, src, ttnn::dtype_size(dtype) * rows * cols, hipMemcpyDeviceToDevice,
                            as_stream(stream)));
    return TTNN_OK;
  });
}

ttnn_status ttnn_level_id(ttnn_plan_t plan, int32_t node, int32_t* out) {
  Plan* P = get(plan);
  return guard(nullptr, [&]() -> ttnn_status {
    if (!P || !out) throw Error{TTNN_E_INVALID, "NULL argument"};
    *out = level_id(*P, node);
    return TTNN_OK;
  });
}

ttnn_status ttnn_reuse_set(ttnn_plan_t plan, int32_t node, int32_t* count, int32_t* ids) {
  Plan* P = get(plan);
  return guard(nullptr, [&]() -> ttnn_status {
    if (!P || !count || !ids) throw Error{TTNN_E_INVALID, "NULL argument"};
    const ttnn::Node& t = P->nodes[level_id(*P, node)];
    int32_t cnt = 0;                             // free modes are no nodes of the caller
    for (int sidx : t.S)
      if (!P->nodes[sidx].ident) ids[cnt++] = P->nodes[sidx].caller;
    *count = cnt;
    return TTNN_OK;
  });
}

ttnn_status ttnn_reset(ttnn_plan_t plan, void* stream) {
  Plan* P = get(plan);
  if (!P) return TTNN_E_INVALID;
  try {
    P->sticky = TTNN_OK;
    (void)hipGetLastError();
    ttnn::zero_accumulators(*P, as_stream(stream));
    TTNN_HIP(hipGetLastError());
    return TTNN_OK;
  } catch (const Error& e) {
    ttnn::set_error(e.msg);
    P->sticky = e.status == TTNN_E_HIP ? TTNN_E_HIP : TTNN_OK;
    return e.status;
  }
}

ttnn_status ttnn_set_rank1_form(ttnn_plan_t plan, int32_t form) {
  Plan* P = get(plan);
  return guard(P, [&]() -> ttnn_status {
    if (!P) throw Error{TTNN_E_INVALID, "plan is NULL"};
    if (form != TTNN_R1_TERMWISE && form != TTNN_R1_GROUPED) throw Error{TTNN_E_INVALID, "bad rank-1 form"};
    P->rank1_form = form;
    return TTNN_OK;
  });
}

ttnn_status ttnn_set_timing(ttnn_plan_t plan, int32_t on) {
  Plan* P = get(plan);
  return guard(P, [&]() -> ttnn_status {
    if (!P) throw Error{TTNN_E_INVALID, "plan is NULL"};
    if (on && !P->sweep_ev[0]) {
      for (hipEvent_t& e : P->sweep_ev) TTNN_HIP(hipEventCreate(&e));
    }
    P->timing = on != 0;
    P->sweep_recorded = false;
    return TTNN_OK;
  });
}

ttnn_status ttnn_sweep_time_ms(ttnn_plan_t plan, float* ms) {
  Plan* P = get(plan);
  return guard(P, [&]() -> ttnn_status {
    if (!P || !ms) throw Error{TTNN_E_INVALID, "plan or ms is NULL"};
    if (!P->timing || !P->sweep_recorded) throw Error{TTNN_E_STATE, "no timed update since ttnn_set_timing"};
    TTNN_HIP(hipEventSynchronize(P->sweep_ev[1]));
    TTNN_HIP(hipEventElapsedTime(ms, P->sweep_ev[0], P->sweep_ev[1]));
    return TTNN_OK;
  });
}

ttnn_status ttnn_sweep_kind(ttnn_plan_t plan, int32_t* kind) {
  Plan* P = get(plan);
  return guard(P, [&]() -> ttnn_status {
    if (!P || !kind) throw Error{TTNN_E_INVALID, "plan or kind is NULL"};
    const auto& F = P->fused;
    *kind = !F.enabled ? 0 : F.tt ? 3 : F.zout ? 2 : 1;
    return TTNN_OK;
  });
}

ttnn_status ttnn_right_sketch_split(int64_t contraction_run, int64_t rows, int64_t runs, int32_t r, int32_t dtype,
                                    size_t scratch_elems, int32_t compute_units, int64_t* nchunks, int64_t* kchunk) {
  return guard(nullptr, [&]() -> ttnn_status {
    if (!nchunks || !kchunk || compute_units < 1) throw Error{TTNN_E_INVALID, "bad argument"};
    if (dtype != TTNN_F64 && dtype != TTNN_F32 && dtype != TTNN_BF16) throw Error{TTNN_E_INVALID, "bad dtype"};
    const ttnn::RightMfmaSplit sp =
        ttnn::right_mfma_split(contraction_run, rows, runs, r, dtype, scratch_elems, compute_units);
    *nchunks = sp.nch;
    *kchunk = sp.kchunk;
    return TTNN_OK;
  });
}

ttnn_status ttnn_chain_head_split(int64_t group_rows, int64_t rows, int32_t k, int32_t dtype, size_t scratch_elems,
                                  int32_t compute_units, int32_t* in_place, int64_t* nchunks, int64_t* kchunk) {
  return guard(nullptr, [&]() -> ttnn_status {
    if (!in_place || !nchunks || !kchunk || compute_units < 1 || k < 1) throw Error{TTNN_E_INVALID, "bad argument"};
    if (dtype != TTNN_F64 && dtype != TTNN_F32 && dtype != TTNN_BF16) throw Error{TTNN_E_INVALID, "bad dtype"};
    const bool inpl = ttnn::chain_head_in_place(rows, k, scratch_elems);
    const size_t room = inpl ? static_cast<size_t>(rows) * static_cast<size_t>(k) : scratch_elems;
    const ttnn::RightMfmaSplit sp = ttnn::right_mfma_split(group_rows, rows, 1, k, dtype, room, compute_units);
    *in_place = inpl ? 1 : 0;
    *nchunks = sp.nch;
    *kchunk = sp.kchunk;
    return TTNN_OK;
  });
}

const char* ttnn_status_string(ttnn_status s) {
  switch (s) {
    case TTNN_OK: return "ok";
    case TTNN_E_INVALID: return "invalid argument";
    case TTNN_E_TREE: return "invalid index tree";
    case TTNN_E_RANGE: return "out of range";
    case TTNN_E_NOMEM: return "out of device memory";
    case TTNN_E_HIP: return "HIP runtime error";
    case TTNN_E_STATE: return "call out of order";
    case TTNN_E_NUMERIC: return "numerical failure";
  }
  return "unknown status";
}

const char* ttnn_last_error(void) { return ttnn::last_error(); }

}  // extern "C"
