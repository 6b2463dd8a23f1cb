// Serving loop: continuous batching of searches over a stream of inserts and
// deletes, with per-search snapshot visibility and admission by device memory
// budget (include/snn.h, snn_serve_run).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "snn_host.h"

using namespace snn;

#define HIP_TRY(ix, call, what)                              \
  do {                                                       \
    hipError_t e__ = (call);                                 \
    if (e__ != hipSuccess) return (ix)->hip_fail(e__, what); \
  } while (0)

namespace {

using Clock = std::chrono::steady_clock;

struct BatchSlot {
  bool busy = false;
  Workspace W;
  DevBuf out;     // ids, scores, counts of the batch
  PinBuf host;    // their host copy
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  uint32_t q0 = 0, q1 = 0, kmax = 0, min_seq = 0;
  uint64_t bytes = 0;
};

struct MutGroup {
  hipEvent_t ev = nullptr;
  std::vector<uint32_t> reqs;  // request indices (for latency)
};

// pinned staging arena for small uploads (slots, ids, sequence numbers, coords)
struct Arena {
  PinBuf pin;
  size_t cursor = 0;
  void *take(snn_index *ix, size_t bytes, hipStream_t s) {
    bytes = (bytes + 255) / 256 * 256;
    if (cursor + bytes > pin.cap) {
      (void)hipStreamSynchronize(s);  // every earlier copy out of the arena has finished
      cursor = 0;
      if (bytes > pin.cap && pin.ensure(bytes, s) != hipSuccess) return nullptr;
    }
    void *p = (char *)pin.p + cursor;
    cursor += bytes;
    (void)ix;
    return p;
  }
};

double pct(std::vector<double> v, double q) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  size_t i = (size_t)std::ceil(q * v.size()) - 1;
  if (i >= v.size()) i = v.size() - 1;
  return v[i];
}

}  // namespace

extern "C" snn_status snn_serve_run(snn_index *ix, const snn_trace *tr, const snn_serve_params *pp, uint32_t *out_ids,
                                    float *out_scores, uint32_t *out_counts, double *out_latency_ms,
                                    snn_serve_report *report) {
  if (!ix || !tr || !pp) return SNN_E_INVALID;
  if (!tr->kind || !tr->arrival_s || !tr->id || !tr->k || !tr->indptr)
    return ix->fail(SNN_E_INVALID, "serve: null trace array");
  if (pp->max_batch == 0 || pp->max_inflight == 0 || pp->max_inflight > 8 || pp->streams == 0 || pp->streams > 4)
    return ix->fail(SNN_E_INVALID, "serve: bad parameters");
  const uint32_t n = tr->n;
  hipStream_t M = ix->stream;

  // ---------------- validate the whole trace first (all-or-nothing) ----------------
  std::vector<uint32_t> sreq, ireq;  // request index of every search / insert
  uint32_t kmax = 1, ndel = 0;
  {
    std::unordered_set<uint32_t> live;
    live.reserve(ix->id2slot.size() * 2 + n);
    ix->id2slot.for_each([&](uint32_t id, uint32_t) { live.insert(id); });
    VecCheck vc;
    vc.stamps = tr->n >= 256 && ix->cfg.dim <= (1u << 20);
    size_t cap_left = ix->free_slots.size() + (ix->cap - ix->next_fresh);
    for (uint32_t r = 0; r < n; ++r) {
      if (r && tr->arrival_s[r] < tr->arrival_s[r - 1]) return ix->fail(SNN_E_INVALID, "serve: arrivals not sorted");
      if (tr->indptr[r + 1] < tr->indptr[r]) return ix->fail(SNN_E_INVALID, "serve: indptr not monotone");
      const uint64_t len = tr->indptr[r + 1] - tr->indptr[r];
      const uint8_t kd = tr->kind[r];
      if (kd == 0 || kd == 1) {
        if (len > (kd == 0 ? (uint64_t)kPrepCap : (uint64_t)ix->cfg.dim))
          return ix->fail(SNN_E_INVALID, "serve: request %u has too many entries", r);
        if (!snn_check_vector(ix, (uint32_t)len, tr->coords + tr->indptr[r], tr->vals + tr->indptr[r], nullptr,
                              nullptr, vc, "serve"))
          return SNN_E_INVALID;
      }
      if (kd == 0) {
        if (tr->k[r] == 0 || tr->k[r] > kMaxK) return ix->fail(SNN_E_INVALID, "serve: k out of range at %u", r);
        kmax = std::max(kmax, tr->k[r]);
        sreq.push_back(r);
      } else if (kd == 1) {
        if (tr->id[r] == 0xFFFFFFFFu || !live.insert(tr->id[r]).second)
          return ix->fail(SNN_E_INVALID, "serve: insert of live id %u at %u", tr->id[r], r);
        ireq.push_back(r);
      } else if (kd == 2) {
        if (!live.erase(tr->id[r])) return ix->fail(SNN_E_INVALID, "serve: delete of id %u that is not live", tr->id[r]);
        ++ndel;
      } else {
        return ix->fail(SNN_E_INVALID, "serve: unknown request kind %u", (unsigned)kd);
      }
    }
    // deleted slots are reused only after the searches that may see them finish,
    // so in the worst case every insert needs a fresh or already-free slot
    if (ireq.size() > cap_left) return ix->fail(SNN_E_FULL, "serve: %zu inserts but %zu free slots", ireq.size(), cap_left);
  }
  const uint32_t nS = (uint32_t)sreq.size();

  // ---------------- inputs into HBM: searches and insert vectors ----------------
  auto upload_csr = [&](const std::vector<uint32_t> &reqs, DevBuf &ptr, DevBuf &c, DevBuf &v,
                        std::vector<uint64_t> &hptr) -> snn_status {
    hptr.assign(reqs.size() + 1, 0);
    for (size_t i = 0; i < reqs.size(); ++i) {
      const uint32_t r = reqs[i];
      uint64_t nz = 0;
      for (uint64_t e = tr->indptr[r]; e < tr->indptr[r + 1]; ++e) nz += tr->vals[e] != 0.0f;
      hptr[i + 1] = hptr[i] + nz;
    }
    const uint64_t tot = hptr.back();
    std::vector<uint32_t> hc(tot);
    std::vector<float> hv(tot);
    for (size_t i = 0; i < reqs.size(); ++i) {
      uint64_t o = hptr[i];
      const uint32_t r = reqs[i];
      for (uint64_t e = tr->indptr[r]; e < tr->indptr[r + 1]; ++e)
        if (tr->vals[e] != 0.0f) {
          hc[o] = tr->coords[e];
          hv[o] = tr->vals[e];
          ++o;
        }
    }
    HIP_TRY(ix, ptr.ensure(hptr.size() * 8, M), "serve upload");
    HIP_TRY(ix, c.ensure(tot * 4 + 16, M), "serve upload");
    HIP_TRY(ix, v.ensure(tot * 4 + 16, M), "serve upload");
    HIP_TRY(ix, hipMemcpy(ptr.p, hptr.data(), hptr.size() * 8, hipMemcpyHostToDevice), "serve upload");
    if (tot) {
      HIP_TRY(ix, hipMemcpy(c.p, hc.data(), tot * 4, hipMemcpyHostToDevice), "serve upload");
      HIP_TRY(ix, hipMemcpy(v.p, hv.data(), tot * 4, hipMemcpyHostToDevice), "serve upload");
    }
    return SNN_OK;
  };
  DevBuf s_ptr, s_c, s_v, s_seq, s_k, i_ptr, i_c, i_v;
  std::vector<uint64_t> hs_ptr, hi_ptr;
  HIP_TRY(ix, hipStreamSynchronize(M), "sync");
  snn_status st = upload_csr(sreq, s_ptr, s_c, s_v, hs_ptr);
  if (st != SNN_OK) return st;
  st = upload_csr(ireq, i_ptr, i_c, i_v, hi_ptr);
  if (st != SNN_OK) return st;
  {
    std::vector<uint32_t> seq(nS), kk(nS);
    for (uint32_t i = 0; i < nS; ++i) {
      seq[i] = sreq[i] + 1;  // sequence numbers start at 1
      kk[i] = tr->k[sreq[i]];
    }
    HIP_TRY(ix, s_seq.ensure((size_t)nS * 4 + 16, M), "serve upload");
    HIP_TRY(ix, s_k.ensure((size_t)nS * 4 + 16, M), "serve upload");
    if (nS) {
      HIP_TRY(ix, hipMemcpy(s_seq.p, seq.data(), (size_t)nS * 4, hipMemcpyHostToDevice), "serve upload");
      HIP_TRY(ix, hipMemcpy(s_k.p, kk.data(), (size_t)nS * 4, hipMemcpyHostToDevice), "serve upload");
    }
  }
  std::vector<uint32_t> ins_index(n, 0), srch_index(n, 0);
  for (uint32_t i = 0; i < (uint32_t)ireq.size(); ++i) ins_index[ireq[i]] = i;
  for (uint32_t i = 0; i < nS; ++i) srch_index[sreq[i]] = i;

  // ---------------- snapshot state ----------------
  HIP_TRY(ix, hipMalloc(&ix->vis, (size_t)ix->cap * 8), "serve visibility");
  HIP_TRY(ix, hipMalloc(&ix->dirty, (size_t)ix->W * 8), "serve visibility");
  HIP_TRY(ix, launch_serve_init(ix->vis, ix->dirty, ix->dev.live, ix->cap, M), "serve init");
  HIP_TRY(ix, hipStreamSynchronize(M), "sync");

  std::vector<hipStream_t> streams(pp->streams, nullptr);
  for (auto &s : streams) HIP_TRY(ix, hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "serve streams");
  std::vector<BatchSlot> slots(pp->max_inflight);
  for (uint32_t i = 0; i < pp->max_inflight; ++i) {
    slots[i].stream = streams[i % streams.size()];
    HIP_TRY(ix, hipEventCreateWithFlags(&slots[i].done, hipEventDisableTiming), "serve events");
  }
  Arena arena;
  HIP_TRY(ix, arena.pin.ensure((size_t)32 << 20, M), "serve staging");

  std::vector<double> lat(nS, 0.0), mlat;
  std::vector<double> arrival(tr->arrival_s, tr->arrival_s + n);
  std::vector<MutGroup> mut_inflight;
  hipEvent_t last_mut = nullptr;  // the latest mutation group's completion
  struct Pending {
    uint32_t slot, dseq;
  };
  std::vector<Pending> pending;  // deleted slots waiting to be reclaimed
  std::vector<std::vector<uint32_t>> pending_coords;

  snn_serve_report R{};
  uint64_t inflight_bytes = 0;
  uint32_t next_req = 0, form_q0 = 0, form_q1 = 0;  // forming batch = searches [form_q0, form_q1)
  uint32_t form_kmax = 0;
  const uint32_t tile_docs_est = (uint32_t)kBlock * ix->tune.R_batch;
  auto batch_bytes = [&](uint32_t q0, uint32_t q1, uint32_t km) -> uint64_t {
    const uint32_t tiles = std::max<uint32_t>(1, (ix->next_fresh + tile_docs_est - 1) / tile_docs_est + 1);
    const uint64_t nq = q1 - q0;
    return nq * tiles * km * 8ull + (hs_ptr[q1] - hs_ptr[q0]) * 16ull + nq * (64ull + tiles * 4ull + km * 8ull);
  };

  const auto t0 = Clock::now();
  auto now_s = [&]() { return std::chrono::duration<double>(Clock::now() - t0).count(); };

  // ---------------- mutations ----------------
  std::vector<uint32_t> g_slots, g_ids, g_seqs, g_reqs;
  auto flush_inserts = [&](uint32_t first_ins) -> snn_status {
    const uint32_t cnt = (uint32_t)g_slots.size();
    if (!cnt) return SNN_OK;
    // slots, ids, sequence numbers, then (forward store) each document's region
    const size_t o_off = ((size_t)cnt * 12 + 7) / 8 * 8;
    const size_t bytes = ix->has_fwd ? o_off + (size_t)cnt * 8 : (size_t)cnt * 12;
    std::vector<uint64_t> doc_off;
    if (ix->has_fwd) {
      doc_off.resize(cnt);
      snn_status fs = ix->fwd_place(g_slots.data(), hi_ptr.data() + first_ins, cnt, doc_off.data());
      if (fs != SNN_OK) return fs;
    }
    uint32_t *hp = (uint32_t *)arena.take(ix, bytes, M);
    if (!hp) return ix->fail(SNN_E_NOMEM, "serve staging");
    memcpy(hp, g_slots.data(), cnt * 4);
    memcpy(hp + cnt, g_ids.data(), cnt * 4);
    memcpy(hp + 2 * cnt, g_seqs.data(), cnt * 4);
    if (ix->has_fwd) memcpy((char *)hp + o_off, doc_off.data(), (size_t)cnt * 8);
    uint32_t *dp = nullptr;
    HIP_TRY(ix, hipMallocAsync((void **)&dp, bytes, M), "serve upload");
    HIP_TRY(ix, hipMemcpyAsync(dp, hp, bytes, hipMemcpyHostToDevice, M), "serve upload");
    HIP_TRY(ix, launch_serve_mark(ix->vis, ix->dirty, cnt, dp, dp + 2 * cnt, 1, M), "serve mark");
    HIP_TRY(ix,
            launch_insert(ix->dev, cnt, dp, dp + cnt, (const uint64_t *)i_ptr.p + first_ins, (const uint32_t *)i_c.p,
                          (const float *)i_v.p, ix->fw, ix->has_fwd ? (const uint64_t *)((char *)dp + o_off) : nullptr,
                          M),
            "serve insert");
    HIP_TRY(ix, hipFreeAsync(dp, M), "serve upload");
    g_slots.clear();
    g_ids.clear();
    g_seqs.clear();
    return SNN_OK;
  };
  auto mark_deletes = [&](const std::vector<uint32_t> &ds, const std::vector<uint32_t> &seqs) -> snn_status {
    const uint32_t cnt = (uint32_t)ds.size();
    if (!cnt) return SNN_OK;
    uint32_t *hp = (uint32_t *)arena.take(ix, (size_t)cnt * 8, M);
    if (!hp) return ix->fail(SNN_E_NOMEM, "serve staging");
    memcpy(hp, ds.data(), cnt * 4);
    memcpy(hp + cnt, seqs.data(), cnt * 4);
    uint32_t *dp = nullptr;
    HIP_TRY(ix, hipMallocAsync((void **)&dp, (size_t)cnt * 8, M), "serve upload");
    HIP_TRY(ix, hipMemcpyAsync(dp, hp, (size_t)cnt * 8, hipMemcpyHostToDevice, M), "serve upload");
    HIP_TRY(ix, launch_serve_mark(ix->vis, ix->dirty, cnt, dp, dp + cnt, 0, M), "serve mark");
    HIP_TRY(ix, hipFreeAsync(dp, M), "serve upload");
    return SNN_OK;
  };
  // clear the postings and live bit of reclaimed slots (their old documents are invisible to
  // every search still in flight), then hand the slots to later inserts
  auto reclaim = [&](uint32_t min_seq) -> snn_status {
    std::vector<uint32_t> sl;
    std::vector<uint64_t> ptr(1, 0);
    std::vector<uint32_t> co;
    size_t keep = 0;
    for (size_t i = 0; i < pending.size(); ++i) {
      if (pending[i].dseq < min_seq) {
        sl.push_back(pending[i].slot);
        co.insert(co.end(), pending_coords[i].begin(), pending_coords[i].end());
        ptr.push_back(co.size());
      } else {
        pending[keep] = pending[i];
        pending_coords[keep].swap(pending_coords[i]);
        ++keep;
      }
    }
    pending.resize(keep);
    pending_coords.resize(keep);
    if (sl.empty()) return SNN_OK;
    const size_t cn = sl.size(), ne = co.size();
    char *hp = (char *)arena.take(ix, cn * 4 + (cn + 1) * 8 + ne * 4 + 16, M);
    if (!hp) return ix->fail(SNN_E_NOMEM, "serve staging");
    const size_t o_ptr = (cn * 4 + 7) / 8 * 8, o_c = o_ptr + (cn + 1) * 8;
    memcpy(hp, sl.data(), cn * 4);
    memcpy(hp + o_ptr, ptr.data(), (cn + 1) * 8);
    if (ne) memcpy(hp + o_c, co.data(), ne * 4);
    char *dp = nullptr;
    HIP_TRY(ix, hipMallocAsync((void **)&dp, o_c + ne * 4 + 16, M), "serve upload");
    HIP_TRY(ix, hipMemcpyAsync(dp, hp, o_c + ne * 4, hipMemcpyHostToDevice, M), "serve upload");
    HIP_TRY(ix,
            launch_delete(ix->dev, (uint32_t)cn, (uint32_t *)dp, (uint64_t *)(dp + o_ptr), (uint32_t *)(dp + o_c), 1, 1,
                          M),
            "serve reclaim");
    HIP_TRY(ix, hipFreeAsync(dp, M), "serve upload");
    for (uint32_t s : sl) ix->free_slots.release(s);
    return SNN_OK;
  };

  // ---------------- the loop ----------------
  st = SNN_OK;
  while (st == SNN_OK) {
    const double now = now_s();
    bool progressed = false;
    // 1. admit arrived requests, in order
    std::vector<uint32_t> del_slots, del_seqs;
    uint32_t first_ins = 0;
    while (next_req < n && (!pp->realtime || arrival[next_req] <= now)) {
      const uint32_t r = next_req;
      const uint8_t kd = tr->kind[r];
      if (kd == 0) {
        const uint32_t qi = srch_index[r];
        const uint32_t km = std::max(form_kmax, tr->k[r]);
        if (form_q1 - form_q0 >= pp->max_batch) break;
        const uint64_t alone = batch_bytes(qi, qi + 1, tr->k[r]);
        if (alone > pp->budget_bytes) {  // can never run: reject
          if (form_q1 == form_q0) {
            if (out_counts) out_counts[qi] = 0xFFFFFFFFu;
            lat[qi] = -1;
            ++R.rejected;
            form_q0 = form_q1 = qi + 1;
            ++next_req;
            progressed = true;
            continue;
          }
          break;  // launch what is formed first
        }
        if (form_q1 > form_q0 && inflight_bytes + batch_bytes(form_q0, qi + 1, km) > pp->budget_bytes) break;
        if (form_q1 == form_q0) form_q0 = qi;
        form_q1 = qi + 1;
        form_kmax = km;
      } else {
        // mutations apply in order; a pending run of inserts is flushed before a delete
        if (kd == 1) {
          if (g_slots.empty()) first_ins = ins_index[r];
          const uint32_t slot = ix->free_slots.take(ix->next_fresh, ix->cap, ix->array_coords > 0);
          const uint32_t id = tr->id[r];
          g_slots.push_back(slot);
          g_ids.push_back(id);
          g_seqs.push_back(r + 1);
          ix->id2slot.put(id, slot);
          ix->slot_id[slot] = id;
          std::vector<uint32_t> &f = ix->fwd[slot];
          f.clear();
          for (uint64_t e = tr->indptr[r]; e < tr->indptr[r + 1]; ++e)
            if (tr->vals[e] != 0.0f) f.push_back(tr->coords[e]);
          ++ix->live;
          ++R.inserts;
        } else {
          // the delete's mark is applied after this admission round's inserts, which
          // is the order that matters: a document inserted and deleted in the same
          // round gets its insert sequence first
          const uint32_t id = tr->id[r];
          const uint32_t slot = *ix->id2slot.find(id);  // validated live above
          ix->id2slot.erase(id);
          ix->slot_id[slot] = 0xFFFFFFFFu;
          del_slots.push_back(slot);
          del_seqs.push_back(r + 1);
          pending.push_back({slot, r + 1});
          pending_coords.push_back(std::move(ix->fwd[slot]));
          ix->fwd[slot] = std::vector<uint32_t>();
          --ix->live;
          ++R.deletes;
        }
        g_reqs.push_back(r);
      }
      ++next_req;
      progressed = true;
    }
    if (st != SNN_OK) break;
    if (!g_slots.empty()) {
      st = flush_inserts(first_ins);
      if (st != SNN_OK) break;
    }
    if (!del_slots.empty()) {
      st = mark_deletes(del_slots, del_seqs);
      if (st != SNN_OK) break;
    }
    if (!g_reqs.empty()) {
      MutGroup g;
      if (hipEventCreateWithFlags(&g.ev, hipEventDisableTiming) != hipSuccess || hipEventRecord(g.ev, M) != hipSuccess) {
        st = ix->fail(SNN_E_DEVICE, "serve: mutation event");
        break;
      }
      g.reqs.swap(g_reqs);
      last_mut = g.ev;
      mut_inflight.push_back(std::move(g));
      ix->mutations++;
    }
    // 2. reclaim deleted slots no search in flight (or forming) can still see
    if (!pending.empty()) {
      uint32_t min_seq = 0xFFFFFFFFu;
      for (auto &b : slots)
        if (b.busy) min_seq = std::min(min_seq, b.min_seq);
      if (form_q1 > form_q0) min_seq = std::min(min_seq, sreq[form_q0] + 1);
      st = reclaim(min_seq);
      if (st != SNN_OK) break;
    }
    // 3. launch the forming batch on a free slot
    if (form_q1 > form_q0) {
      BatchSlot *b = nullptr;
      for (auto &x : slots)
        if (!x.busy) {
          b = &x;
          break;
        }
      const uint64_t bytes = batch_bytes(form_q0, form_q1, form_kmax);
      if (b && inflight_bytes + bytes <= pp->budget_bytes) {
        const uint32_t nq = form_q1 - form_q0, km = form_kmax;
        if (last_mut && hipStreamWaitEvent(b->stream, last_mut, 0) != hipSuccess) {
          st = ix->fail(SNN_E_DEVICE, "serve: wait event");
          break;
        }
        if (b->out.ensure((size_t)nq * km * 8 + (size_t)nq * 4 + 256, b->stream) != hipSuccess ||
            b->host.ensure((size_t)nq * km * 8 + (size_t)nq * 4 + 256, b->stream) != hipSuccess) {
          st = ix->fail(SNN_E_NOMEM, "serve: batch buffers");
          break;
        }
        uint32_t *ids = (uint32_t *)b->out.p;
        float *sc = (float *)(ids + (size_t)nq * km);
        uint32_t *cnt = (uint32_t *)(sc + (size_t)nq * km);
        SearchOpts o;
        o.kq = (const uint32_t *)s_k.p + form_q0;
        o.qseq = (const uint32_t *)s_seq.p + form_q0;
        o.ebase = hs_ptr[form_q0];
        o.wsp = &b->W;
        o.no_graph = true;
        st = ix->run_search(nq, (const uint64_t *)s_ptr.p + form_q0, hs_ptr[form_q1], (const uint32_t *)s_c.p,
                            (const float *)s_v.p, km, SNN_MODE_BATCHED, ids, sc, cnt, b->stream, o);
        if (st != SNN_OK) break;
        if (hipMemcpyAsync(b->host.p, b->out.p, (size_t)nq * km * 8 + (size_t)nq * 4, hipMemcpyDeviceToHost,
                           b->stream) != hipSuccess ||
            hipEventRecord(b->done, b->stream) != hipSuccess) {
          st = ix->fail(SNN_E_DEVICE, "serve: batch readback");
          break;
        }
        b->busy = true;
        b->q0 = form_q0;
        b->q1 = form_q1;
        b->kmax = km;
        b->min_seq = sreq[form_q0] + 1;
        b->bytes = bytes;
        inflight_bytes += bytes;
        R.peak_workspace_bytes = std::max<uint64_t>(R.peak_workspace_bytes, inflight_bytes);
        R.batches++;
        R.max_batch_seen = std::max(R.max_batch_seen, nq);
        uint32_t busy = 0;
        for (auto &x : slots) busy += x.busy;
        R.max_inflight_seen = std::max(R.max_inflight_seen, busy);
        form_q0 = form_q1;
        form_kmax = 0;
        progressed = true;
      }
    }
    // 4. completions
    for (auto &b : slots) {
      if (!b.busy) continue;
      hipError_t q = hipEventQuery(b.done);
      if (q == hipErrorNotReady) continue;
      if (q != hipSuccess) {
        st = ix->hip_fail(q, "serve: batch");
        break;
      }
      const double t = now_s();
      const uint32_t nq = b.q1 - b.q0, km = b.kmax;
      const uint32_t *hid = (const uint32_t *)b.host.p;
      const float *hsc = (const float *)(hid + (size_t)nq * km);
      const uint32_t *hcnt = (const uint32_t *)(hsc + (size_t)nq * km);
      for (uint32_t i = 0; i < nq; ++i) {
        const uint32_t qi = b.q0 + i;
        lat[qi] = (t - (pp->realtime ? arrival[sreq[qi]] : 0.0)) * 1000.0;
        if (out_counts) out_counts[qi] = hcnt[i];
        if (out_ids) memcpy(out_ids + (size_t)qi * kmax, hid + (size_t)i * km, (size_t)std::min(hcnt[i], km) * 4);
        if (out_scores) memcpy(out_scores + (size_t)qi * kmax, hsc + (size_t)i * km, (size_t)std::min(hcnt[i], km) * 4);
      }
      inflight_bytes -= b.bytes;
      b.busy = false;
      progressed = true;
    }
    if (st != SNN_OK) break;
    for (size_t i = 0; i < mut_inflight.size();) {
      hipError_t q = hipEventQuery(mut_inflight[i].ev);
      if (q == hipErrorNotReady) {
        ++i;
        continue;
      }
      const double t = now_s();
      for (uint32_t r : mut_inflight[i].reqs) mlat.push_back((t - (pp->realtime ? arrival[r] : 0.0)) * 1000.0);
      if (mut_inflight[i].ev == last_mut) last_mut = nullptr;
      (void)hipEventDestroy(mut_inflight[i].ev);
      mut_inflight.erase(mut_inflight.begin() + i);
      progressed = true;
    }
    bool busy = false;
    for (auto &b : slots) busy |= b.busy;
    if (next_req >= n && !busy && form_q1 == form_q0 && mut_inflight.empty()) break;
    if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
  const double wall = now_s();

  // ---------------- wind down: finish, reclaim everything, leave serving mode ----------------
  (void)hipStreamSynchronize(M);
  for (auto &b : slots) {
    if (b.stream) (void)hipStreamSynchronize(b.stream);
  }
  if (st == SNN_OK) st = reclaim(0xFFFFFFFFu);
  (void)hipStreamSynchronize(M);
  for (auto &g : mut_inflight) (void)hipEventDestroy(g.ev);
  for (auto &b : slots) {
    (void)hipEventDestroy(b.done);
    b.W.release();
    b.out.release();
    b.host.release();
  }
  for (auto &s : streams) (void)hipStreamDestroy(s);
  (void)hipFree(ix->vis);
  (void)hipFree(ix->dirty);
  ix->vis = nullptr;
  ix->dirty = nullptr;
  arena.pin.release();
  if (st != SNN_OK) return st;

  std::vector<double> ok;
  for (double v : lat)
    if (v >= 0) ok.push_back(v);
  R.searches = nS;
  R.wall_s = wall;
  R.search_qps = wall > 0 ? (nS - R.rejected) / wall : 0;
  R.p50_ms = pct(ok, 0.50);
  R.p90_ms = pct(ok, 0.90);
  R.p99_ms = pct(ok, 0.99);
  R.max_ms = ok.empty() ? 0 : *std::max_element(ok.begin(), ok.end());
  double sum = 0;
  for (double v : ok) sum += v;
  R.mean_ms = ok.empty() ? 0 : sum / ok.size();
  R.mutation_p50_ms = pct(mlat, 0.50);
  R.mutation_p99_ms = pct(mlat, 0.99);
  if (out_latency_ms)
    for (uint32_t i = 0; i < nS; ++i) out_latency_ms[i] = lat[i];
  if (report) *report = R;
  (void)ndel;
  return SNN_OK;
}
