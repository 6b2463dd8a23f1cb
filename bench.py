#!/usr/bin/env python3
"""Sinnamon search throughput on one MI355X.

Workload (synthetic, seeded): 1,000,000 SPLADE-shaped documents over dim 30,522
(nnz lognormal with mean 120, Zipf(1.05) coordinates, Exp(1) values), 1,024
queries (nnz lognormal mean 40), sketch m = 128 buckets per half, h = 1, k = 10.
A step is one pass of the whole search path (query preparation, scoring,
top-k selection, merge) over the batch of 1,024 queries, with the inputs
already in HBM. Forms: plain (one query at a time) and batched (one persistent
launch per batch). `value` is the best form's queries/s.

Also reported: the roofline of the scoring kernel (algorithmic bytes per query
as defined in the design notes, over its measured launch time), recall@10 of
the approximate results against exact brute force, and the FP64 oracle timed
on the host's cores on a bounded query sample.

Progress goes to stderr; stdout gets exactly one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "queries/s at fixed recall@10 (1M docs) + HBM GB/s; learned/batched vs plain; p99"
HBM_PEAK_GBS = 8000.0
# VALU issue peak: 256 CUs x 4 SIMDs, each retiring one wave64 instruction per
# 4 cycles (16 lanes a cycle) at 2.4 GHz, in lane operations per second (1e12)
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12


def log(*a):
    print("[bench %7.1fs]" % (time.time() - T0), *a, file=sys.stderr, flush=True)


T0 = time.time()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--docs", type=int, default=1_000_000)
    ap.add_argument("--queries", type=int, default=1024)
    ap.add_argument("--k", type=int, default=10)
    ap.add_argument("--forms", default="plain,batched,learned")
    ap.add_argument("--train-queries", type=int, default=50000)
    ap.add_argument("--filter-fallback", type=float, default=0.01,
                    help="share of held-out queries whose predicted threshold may exceed their k-th score")
    ap.add_argument("--no-small", action="store_true", help="skip the learned-filter workload on the 10k-doc index")
    ap.add_argument("--no-batch4m", action="store_true", help="skip the 4M-doc batching workload")
    ap.add_argument("--no-serving", action="store_true", help="skip the 8M-capacity serving workload")
    ap.add_argument("--kprimes", default="10,100,300,500,1000,4096",
                    help="k' values of the re-ranking (Alg. 7) forms on the 1M-doc index; empty to skip")
    ap.add_argument("--no-g100", action="store_true", help="skip the G100 workload of the paper (Section 6.5)")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the bfloat16 / upper-only sketch variants of the 1M-doc index")
    ap.add_argument("--no-g200", action="store_true", help="skip the G200 workload of the paper (Section 6.5)")
    ap.add_argument("--anytime", default="5,10,20",
                    help="coordinate budgets of the anytime re-ranking forms (k' = 1000); empty to skip")
    ap.add_argument("--serving-ops", type=int, default=100_000)
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--cpu-sample", type=int, default=64, help="queries checked against the oracle's Alg. 7")
    ap.add_argument("--cpu-sample-one", type=int, default=64, help="queries timed on one host thread")
    ap.add_argument("--cpu-reps", type=int, default=5, help="runs of the all-thread oracle timing (median)")
    ap.add_argument("--updates", type=int, default=131072,
                    help="documents deleted and re-inserted to time the update kernels (0: build only)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compact", action="store_true",
                    help="leave every coordinate in its bitmap container (no array containers)")
    ap.add_argument("--schedule", default="",
                    help="R,Q,grid,persistent: the batched schedule to use instead of autotuning (profiling runs)")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="MiB: run one plain device copy of this size first (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only (the index is not sharded across GPUs); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2301_10622_amd as P
    from synth import gen

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.calibrate_copy:
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: %d bytes read, %d bytes written" % (nbytes, nbytes))
        del src, dst
    log("generating workload")
    w = gen.make_splade_like(0, docs=args.docs, queries=args.queries)
    log("docs %d (nnz %d), queries %d (nnz %d)" % (w.docs.rows, w.docs.nnz, w.queries.rows, w.queries.nnz))

    stream = torch.cuda.Stream()  # non-default stream (HIP graphs cannot capture the legacy stream)
    torch.cuda.set_stream(stream)
    # the forward store (vector storage of Alg. 7) serves the re-ranking forms;
    # the Sinnamon search itself never reads it
    ix = P.Index(w.n, w.m, w.h, capacity=w.docs.rows, hash_seed=w.hash_seed, stream=stream, forward_store=True)
    torch.cuda.synchronize()
    ix.profile(True)
    t = time.time()
    P.load_docs(ix, w.docs, compact=False)
    torch.cuda.synchronize()
    t_ins = time.time() - t
    build_upd = ix.profile_read_updates()
    containers = {"compacted": not args.no_compact}
    if not args.no_compact:
        t = time.time()
        ix.compact()
        t_compact = time.time() - t
        cls = ix.container_classes()
        ll = np.bincount(w.docs.coords, minlength=w.n).astype(np.int64)
        nap = int(ll[cls != 0].sum())
        nrows = int(np.count_nonzero((cls != 0) & (ll > 0)))
        nblk = -(-w.docs.rows // 16384) * 16
        # offsets (2 bytes) and both bounds (4 bytes each) per array posting, and the block-offset rows
        cbytes = nap * (2 + 4 + 4) + (nrows + 1) * (nblk + 1) * 4
        containers.update({"compaction_s": round(t_compact, 4), "array_coords": int(cls.sum()), "dim": w.n,
                           "query_entries_with_arrays": round(float(cls[w.queries.coords].mean()), 4),
                           "array_postings": nap, "all_postings": int(ll.sum()), "container_bytes": cbytes})
        log("compaction %.3fs: %d of %d coordinates with array containers" % (t_compact, int(cls.sum()), w.n))
    ix.profile(False)
    log("index built: %.2fs (%.0f docs/s through the host API; insert kernel %.2f ms for %d docs)" % (
        t_ins, w.docs.rows / t_ins, build_upd["insert_ms"], build_upd["insert_docs"]))

    # algorithmic bytes per query: every posting of a query coordinate costs its
    # 4-byte id and h 4-byte sketch values; plus 12 B per query entry and 8 B per result
    list_len = np.bincount(w.docs.coords, minlength=w.n).astype(np.int64)
    qptr = w.queries.indptr
    postings = np.add.reduceat(list_len[w.queries.coords], qptr[:-1]) if w.queries.nnz else np.zeros(w.queries.rows)
    postings = np.where(np.diff(qptr) > 0, postings, 0)
    psi_q = np.diff(qptr)

    def alg_bytes(k):
        return float((postings * (4 + 4 * w.h) + 12 * psi_q + 8 * k).sum())

    ip = torch.tensor(w.queries.indptr, dtype=torch.int64, device=dev)
    qc = torch.tensor(w.queries.coords.astype(np.int32), device=dev)
    qv = torch.tensor(w.queries.vals, device=dev)
    nq = w.queries.rows
    total = int(w.queries.nnz)

    def run_form(mode, k, steps, warmup):
        out = (torch.empty((nq, k), dtype=torch.int32, device=dev), torch.empty((nq, k), dtype=torch.float32, device=dev),
               torch.empty(nq, dtype=torch.int32, device=dev))
        for _ in range(warmup):
            ix.search_batch_dev(ip, qc, qv, k, mode=mode, out=out, total=total)
        # timed region 1: throughput (batched forms replay a captured HIP graph)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ix.search_batch_dev(ip, qc, qv, k, mode=mode, out=out, total=total)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        # timed region 2: the same steps launched eagerly with HIP events
        # bracketing every launch of the scoring kernel on its stream
        ix.profile(True)
        ix.profile_read()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(steps):
            ix.search_batch_dev(ip, qc, qv, k, mode=mode, out=out, total=total)
        torch.cuda.synchronize()
        dt_eager = time.perf_counter() - t1
        kms, launches = ix.profile_read()
        ix.profile(False)
        ms_step = dt * 1000.0 / steps
        res = {"qps": nq / (ms_step / 1000.0), "ms_per_step": ms_step, "steps": steps,
               "ms_per_step_eager_profiled": dt_eager * 1000.0 / steps,
               "tile_kernel_ms_per_launch": kms / max(launches, 1), "tile_launches_per_step": launches / steps}
        return res, out

    if args.schedule:
        R, Q, grid, pers = [int(x) for x in args.schedule.split(",")]
        ix.set_schedule(16, R, grid, bool(pers), Q)
        sched = ix.schedule()
    else:
        log("autotuning the schedule on the batch")
        sched = ix.autotune(ip, qc, qv, args.k, total=total)
    log("schedule: %s" % sched)

    forms = {}
    outs = {}
    filters = {}
    for name in args.forms.split(","):
        mode = {"plain": P.MODE_PLAIN, "batched": P.MODE_BATCHED, "learned": P.MODE_LEARNED}[name]
        for k in (args.k, 100):
            steps = args.plain_steps if name == "plain" else args.steps
            warm = 1 if name == "plain" else args.warmup
            if name == "learned":
                # the filter predicts the k-th score: train one for this k on
                # separate training queries (labels from the plain method)
                tq = gen.make_splade_like(2, docs=0, queries=args.train_queries).queries
                tt = (torch.tensor(tq.indptr, dtype=torch.int64, device=dev),
                      torch.tensor(tq.coords.astype(np.int32), device=dev), torch.tensor(tq.vals, device=dev))
                rep = ix.filter_train(*tt, k=k, epochs=8, batch=512, lr=1e-3, total=int(tq.nnz),
                                      target_fallback=args.filter_fallback)
                filters["k%d" % k] = {kk: (round(v, 4) if isinstance(v, float) else v) for kk, v in rep.items()}
                log("filter k=%d trained: %s" % (k, filters["k%d" % k]))
                del tt
            r, out = run_form(mode, k, steps, warm)
            if name == "learned":
                r["fallbacks_last_step"] = ix.last_batch_status()[1]
            ab = alg_bytes(k)
            r["alg_bytes_per_step"] = ab
            r["alg_GBps"] = ab / (r["ms_per_step"] / 1000.0) / 1e9
            forms["%s_k%d" % (name, k)] = r
            outs[(name, k)] = out
            log("%-8s k=%-4d %8.3f ms/step  %10.0f q/s  tile kernel %.3f ms x %.0f/step  alg %.0f GB/s" % (
                name, k, r["ms_per_step"], r["qps"], r["tile_kernel_ms_per_launch"], r["tile_launches_per_step"],
                r["alg_GBps"]))

    # ranking with k' >= k (Alg. 7): Sinnamon candidates, exact re-rank from HBM
    # and the anytime variant (a coordinate budget c in the order of Alg. 6) at k' = 1000
    rerank = {}
    kprimes = [int(x) for x in args.kprimes.split(",") if x.strip()]
    budgets = [int(x) for x in args.anytime.split(",") if x.strip()]
    variants = [(kp, 0) for kp in kprimes] + [(1000, c) for c in budgets]
    for kp, c in variants:
        out = (torch.empty((nq, args.k), dtype=torch.int32, device=dev),
               torch.empty((nq, args.k), dtype=torch.float32, device=dev), torch.empty(nq, dtype=torch.int32, device=dev))
        for _ in range(args.warmup):
            ix.search_ex_dev(ip, qc, qv, args.k, k_prime=kp, max_coords=c, out=out, total=total)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ix.search_ex_dev(ip, qc, qv, args.k, k_prime=kp, max_coords=c, out=out, total=total)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1000.0 / args.steps
        rerank[(kp, c)] = {"qps": nq / (ms / 1000.0), "ms_per_step": ms, "steps": args.steps}
        outs[("rerank", kp, c)] = out
        log("rerank   k=%d k'=%-5d coords %-4s %8.3f ms/step  %10.0f q/s" % (args.k, kp, c or "all", ms,
                                                                          nq / (ms / 1000.0)))

    # the headline index's container classes and mappings (for the compulsory bytes)
    main_classes = ix.container_classes()
    main_buckets = ix.bucket_table().reshape(w.h, w.n)

    # the learned filter starting the selection of the k' = 1,000 candidates of
    # Alg. 7 in place of the sampled first pass (a filter trained for k = k')
    learned_rr = {}
    if "learned" in args.forms.split(",") and 1000 in kprimes:
        tq = gen.make_splade_like(2, docs=0, queries=args.train_queries).queries
        tt = (torch.tensor(tq.indptr, dtype=torch.int64, device=dev),
              torch.tensor(tq.coords.astype(np.int32), device=dev), torch.tensor(tq.vals, device=dev))
        rep = ix.filter_train(*tt, k=1000, epochs=8, batch=512, lr=1e-3, total=int(tq.nnz),
                              target_fallback=args.filter_fallback)
        del tt
        filters["k1000"] = {kk: (round(v, 4) if isinstance(v, float) else v) for kk, v in rep.items()}
        out = (torch.empty((nq, args.k), dtype=torch.int32, device=dev),
               torch.empty((nq, args.k), dtype=torch.float32, device=dev), torch.empty(nq, dtype=torch.int32, device=dev))
        for _ in range(args.warmup):
            ix.search_ex_dev(ip, qc, qv, args.k, mode=P.MODE_LEARNED, k_prime=1000, out=out, total=total)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ix.search_ex_dev(ip, qc, qv, args.k, mode=P.MODE_LEARNED, k_prime=1000, out=out, total=total)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1000.0 / args.steps
        fb = ix.last_batch_status()[1]
        ref = outs[("rerank", 1000, 0)]
        same = all(bool(torch.equal(a, b)) for a, b in zip(out, ref))
        learned_rr = {"qps": nq / (ms / 1000.0), "ms_per_step": ms, "steps": args.steps, "fallbacks_last_step": fb,
                      "identical_to_batched_rerank": same}
        log("learned  k=%d k'=1000 %8.3f ms/step  %10.0f q/s  fallbacks %d  identical to the batched re-rank %s" % (
            args.k, ms, nq / (ms / 1000.0), fb, same))

    # the same batch through the host-buffer call (host validation, upload over
    # PCIe, the batched search, results back): context, never the headline
    qh = w.queries
    host_ids = ix.search_batch(qh.indptr, qh.coords, qh.vals, args.k)[0]
    torch.cuda.synchronize()
    t = time.perf_counter()
    host_reps = 5
    for _ in range(host_reps):
        ix.search_batch(qh.indptr, qh.coords, qh.vals, args.k)
    host_ms = (time.perf_counter() - t) * 1000.0 / host_reps
    ref_form = next((n for n in ("batched", "plain", "learned") if (n, args.k) in outs), None)
    host_api = {"qps": round(nq / (host_ms / 1000.0), 1), "ms_per_batch": round(host_ms, 3),
                "same_ids_as_device_form": None if ref_form is None else bool(np.array_equal(
                    host_ids.astype(np.int64), outs[(ref_form, args.k)][0].cpu().numpy().astype(np.int64)))}
    log("host API  k=%d   %8.3f ms / %d queries  %10.0f q/s (inputs from host memory, results back)" % (
        args.k, host_ms, nq, host_api["qps"]))

    # update kernels (Alg. 5 insert, Section 4.3 delete), timed with HIP events
    # around each launch: the 1M-doc build into fresh slots above, then a delete
    # and re-insert of the first 131,072 documents into the freed slots
    updates = update_kernels(P, np, ix, w, build_upd, args.updates)

    # memory levers: the same collection with a bfloat16 and / or upper-only sketch
    variants_res = {}
    if not args.no_variants:
        ix.close()
        torch.cuda.empty_cache()
        for vname, bf, up, hv in (("bf16", True, False, w.h), ("upper_only", False, True, w.h),
                                  ("bf16_upper_only", True, True, w.h), ("h2", False, False, 2)):
            vx = P.Index(w.n, w.m, hv, capacity=w.docs.rows, hash_seed=w.hash_seed, stream=stream,
                         forward_store=True, sketch_bf16=bf, upper_only=up)
            P.load_docs(vx, w.docs, compact=not args.no_compact)
            # several queries per workgroup need h = 1
            vx.set_schedule(sched["R_plain"], max(16, sched["R_batch"]) if hv != 1 else sched["R_batch"],
                            sched["grid"], bool(sched["persistent"]), sched["qgroup"] if hv == 1 else 1)
            r = {"sketch_bytes": w.m * w.docs.rows * (2 if bf else 4) * (1 if up else 2), "h": hv}
            for form, kw in (("batched_k10", dict(k_prime=0, max_coords=0)),
                             ("rerank_k1000_coords10", dict(k_prime=1000, max_coords=10))):
                out = (torch.empty((nq, args.k), dtype=torch.int32, device=dev),
                       torch.empty((nq, args.k), dtype=torch.float32, device=dev),
                       torch.empty(nq, dtype=torch.int32, device=dev))
                for _ in range(args.warmup):
                    vx.search_ex_dev(ip, qc, qv, args.k, out=out, total=total, **kw)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(args.steps):
                    vx.search_ex_dev(ip, qc, qv, args.k, out=out, total=total, **kw)
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t0) * 1000.0 / args.steps
                r[form] = {"qps": nq / (ms / 1000.0), "ms_per_step": ms}
                outs[("variant", vname, form)] = out
                log("variant %-16s %-22s %8.3f ms/step  %10.0f q/s" % (vname, form, ms, nq / (ms / 1000.0)))
            variants_res[vname] = r
            vx.close()
            torch.cuda.empty_cache()

    # the headline form: the fastest at the headline k
    cand = {n: forms["%s_k%d" % (n, args.k)] for n in args.forms.split(",")}
    best = max(cand, key=lambda n: cand[n]["qps"])
    head = cand[best]
    launch_ms = head["tile_kernel_ms_per_launch"]
    per_launch_queries = nq / head["tile_launches_per_step"]
    ab_launch = alg_bytes(args.k) * per_launch_queries / nq
    kname = tile_kernel_name(sched, best)
    ctr = measured_counters(kname, args.k)
    traffic = ctr.get("traffic_bytes_per_launch") if ctr else None
    comp = compulsory_bytes(np, w, main_classes, list_len, main_buckets)
    comp_launch = comp * per_launch_queries / nq
    launch_s = launch_ms / 1000.0
    if ctr and ctr.get("valu_insts_per_launch"):
        # the bound the kernel reaches: VALU issue (one wave instruction per
        # SIMD every 4 cycles, i.e. 16 lane operations per SIMD and cycle)
        achieved = ctr["valu_insts_per_launch"] * 64 / launch_s / 1e12
        roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": VALU_PEAK_TOPS,
                    "unit": "T VALU lane-ops/s", "frac": round(achieved / VALU_PEAK_TOPS, 4), "traffic": traffic,
                    "valu_insts_per_launch": ctr["valu_insts_per_launch"]}
    else:
        # counters not taken on this kernel source: the compulsory bytes of the
        # launch against the HBM peak
        achieved = comp_launch / launch_s / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic}
    roofline.update({"kernel": kname, "launch_ms": launch_ms, "counters_match_source": bool(ctr),
                     "compulsory_bytes_per_launch": comp_launch,
                     "compulsory_GBps": round(comp_launch / launch_s / 1e9, 1),
                     "alg_bytes_per_launch": ab_launch,
                     "alg_GBps_effective": round(ab_launch / launch_s / 1e9, 1)})
    if traffic:
        roofline["traffic_GBps"] = round(traffic / launch_s / 1e9, 1)
        roofline["hbm_frac_traffic"] = round(traffic / launch_s / 1e9 / HBM_PEAK_GBS, 4)
        roofline["traffic_over_compulsory"] = round(traffic / comp_launch, 3)
    # what this machine's HBM delivers to a plain device copy, beside the published peak
    roofline["copy_GBps"] = round(measured_copy_gbps(torch, dev), 1)

    result = {
        "metric": METRIC, "value": round(head["qps"], 1), "unit": "queries/s", "n_gpus": 1,
        "steps": head["steps"], "warmup": args.warmup, "ms_per_step": round(head["ms_per_step"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name, "docs": w.docs.rows, "dim": w.n, "queries_per_step": nq, "k": args.k,
                   "m": w.m, "h": w.h, "form": best},
        "roofline": roofline,
        "forms": {n: {kk: (round(v, 4) if isinstance(v, float) else v) for kk, v in r.items()} for n, r in forms.items()},
        "insert_docs_per_s_host_api": round(w.docs.rows / t_ins, 1),
        "update_kernels": updates,
        "host_api_search": host_api,
        "containers": containers,
        "schedule": sched,
        "filters": filters,
    }

    # ---------------------------------------------------------------- oracle
    if not args.no_cpu_baseline:
        from oracle import oracle as O

        # timed: every query of the batch on all host threads (median of
        # cpu_reps runs) and a bounded sample on one thread (median of 3);
        # recall over every query, the re-rank agreement on a sample
        S = min(args.cpu_sample, nq)
        sample = w.queries.take(range(S))
        log("oracle: building FP64 index")
        t = time.time()
        ora = O.Index(w.docs, w.n, w.m, w.h, w.hash_seed)
        t_build = time.time() - t
        threads = O.max_threads()
        log("oracle: index %.1fs; timing %d queries on %d threads x %d runs" % (t_build, nq, threads, args.cpu_reps))
        runs = []
        for _ in range(args.cpu_reps):
            t = time.perf_counter()
            oids, osc, oab, ocnt = ora.search(w.queries, args.k, threads=threads)
            runs.append(time.perf_counter() - t)
        t_est = float(np.median(runs))
        t = time.perf_counter()
        eids, esc, _, ecnt = ora.search(w.queries, args.k, exact=True, threads=threads)
        t_exact = time.perf_counter() - t
        S1 = min(args.cpu_sample_one, nq)
        one = []
        for _ in range(3):
            t = time.perf_counter()
            ora.search(w.queries.take(range(S1)), args.k, threads=1)
            one.append(time.perf_counter() - t)
        t_one = float(np.median(one))
        gids = outs[(best, args.k)][0].cpu().numpy().astype(np.int64)
        gcnt = outs[(best, args.k)][2].cpu().numpy()
        rec = []
        agree = []
        for i in range(nq):
            g = set(gids[i][: gcnt[i]].tolist())
            rec.append(len(g & set(eids[i][: ecnt[i]].tolist())) / max(1, min(args.k, ecnt[i])))
            agree.append(len(g & set(oids[i][: ocnt[i]].tolist())) / max(1, ocnt[i]))
        result["recall_at_%d" % args.k] = round(float(np.mean(rec)), 4)
        for fname, r in result["forms"].items():
            if fname.endswith("_k%d" % args.k):
                r["recall_at_%d" % args.k] = result["recall_at_%d" % args.k]
        for vname, r in variants_res.items():
            for form in ("batched_k10", "rerank_k1000_coords10"):
                g_ids = outs[("variant", vname, form)][0].cpu().numpy().astype(np.int64)
                g_cnt = outs[("variant", vname, form)][2].cpu().numpy()
                rr = [len(set(g_ids[i][: g_cnt[i]].tolist()) & set(eids[i][: ecnt[i]].tolist()))
                      / max(1, min(args.k, ecnt[i])) for i in range(nq)]
                r[form]["recall_at_%d" % args.k] = round(float(np.mean(rr)), 4)
        # re-ranked forms: recall against exact brute force (every query),
        # agreement with the oracle's Alg. 7 (the sample)
        for kp, c in variants:
            rids, _, _, rcnt = ora.rerank(sample, args.k, kp, threads=threads, max_coords=c)
            g_ids = outs[("rerank", kp, c)][0].cpu().numpy().astype(np.int64)
            g_cnt = outs[("rerank", kp, c)][2].cpu().numpy()
            rr = [len(set(g_ids[i][: g_cnt[i]].tolist()) & set(eids[i][: ecnt[i]].tolist()))
                  / max(1, min(args.k, ecnt[i])) for i in range(nq)]
            same = [np.array_equal(g_ids[i][: g_cnt[i]], rids[i][: rcnt[i]].astype(np.int64)) for i in range(S)]
            rerank[(kp, c)]["recall_at_%d" % args.k] = round(float(np.mean(rr)), 4)
            rerank[(kp, c)]["identical_to_oracle_alg7"] = round(float(np.mean(same)), 4)
            log("rerank k'=%d coords %s: recall@%d %.4f, identical to the oracle on %.0f%% of %d queries" % (
                kp, c or "all", args.k, np.mean(rr), 100 * np.mean(same), S))
        # recall@100 of the k = 100 forms (identical results in every form)
        ref100 = next(((n, 100) for n in ("batched", "plain", "learned") if (n, 100) in outs), None)
        if ref100 and args.k != 100:
            e100, _, _, c100 = ora.search(w.queries, 100, exact=True, threads=threads)
            g_ids = outs[ref100][0].cpu().numpy().astype(np.int64)
            g_cnt = outs[ref100][2].cpu().numpy()
            r100 = float(np.mean([len(set(g_ids[i][: g_cnt[i]].tolist()) & set(e100[i][: c100[i]].tolist()))
                                  / max(1, min(100, c100[i])) for i in range(nq)]))
            for fname, r in result["forms"].items():
                if fname.endswith("_k100"):
                    r["recall_at_100"] = round(r100, 4)
        result["cpu_baseline"] = {"value": round(nq / t_est, 2), "unit": "queries/s", "cores": threads,
                                  "kind": "oracle",
                                  "sample": "all %d queries of the batch, k=%d, FP64 coordinate-at-a-time estimate "
                                            "+ FindLargest, median of %d runs on %d threads; index build %.1fs "
                                            "excluded" % (nq, args.k, args.cpu_reps, threads, t_build),
                                  "runs_s": [round(x, 3) for x in runs],
                                  "exact_brute_force_qps": round(nq / t_exact, 2),
                                  "single_thread_qps": round(S1 / t_one, 2),
                                  "single_thread_sample": "first %d queries, median of 3 runs" % S1,
                                  "host": host_cpu()}
        log("oracle: %.2f q/s (estimate, median of %d), %.2f q/s (exact), %.2f q/s on one thread; recall@%d %.4f" % (
            nq / t_est, args.cpu_reps, nq / t_exact, S1 / t_one, args.k, result["recall_at_%d" % args.k]))
    if variants_res:
        result["sketch_variants"] = {v: {f: ({kk: (round(x, 4) if isinstance(x, float) else x) for kk, x in d.items()}
                                             if isinstance(d, dict) else d) for f, d in r.items()}
                                     for v, r in variants_res.items()}
    if learned_rr:
        if (1000, 0) in rerank and "recall_at_%d" % args.k in rerank[(1000, 0)]:
            learned_rr["recall_at_%d" % args.k] = rerank[(1000, 0)]["recall_at_%d" % args.k]
        learned_rr["learned_over_batched"] = round(learned_rr["qps"] / rerank[(1000, 0)]["qps"], 4)
        result["learned_rerank_k1000"] = _rounded(learned_rr)
    if rerank:
        result["rerank"] = {("k'=%d" % kp) + ("" if not c else " coords=%d" % c):
                            {kk: (round(v, 4) if isinstance(v, float) else v) for kk, v in r.items()}
                            for (kp, c), r in rerank.items()}
        ok = [v for v in variants if rerank[v].get("recall_at_%d" % args.k, 0) >= 0.9]
        if ok:
            kp, c = max(ok, key=lambda v: rerank[v]["qps"])
            result["at_recall_0.9"] = {"form": "rerank", "k_prime": kp, "max_coords": c,
                                       "qps": round(rerank[(kp, c)]["qps"], 1),
                                       "recall_at_%d" % args.k: rerank[(kp, c)]["recall_at_%d" % args.k]}
    if args.no_variants:
        ix.close()
    if not args.no_small:
        result["learned_small"] = small_learned(args, dev, P, gen, np, torch)
    if not args.no_batch4m:
        result["batch_4m"] = batch_4m(args, dev, P, gen, np, torch)
    if not args.no_g100:
        result["g100"] = paper_gaussian(args, dev, P, gen, np, torch, 100)
    if not args.no_g200:
        result["g200"] = paper_gaussian(args, dev, P, gen, np, torch, 200)
    if not args.no_serving:
        result["serving_8m"] = serving_8m(args, dev, P, gen, np, torch)
    print(json.dumps(result), flush=True)


def host_cpu():
    """The host's CPU model and logical CPU count (as lscpu and nproc give them)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count(),
            "usable_cpus": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()}


def update_kernels(P, np, ix, w, build, n_upd):
    """Docs/s and algorithmic GB/s of the insert and delete kernels.

    Algorithmic bytes per document (Alg. 5 / Section 4.3): insert reads its
    psi_d (coordinate, value) pairs (8 B each) and writes the 2m-entry sketch
    column (4 B each), 8 psi_d + 8m; counted in full it also appends the slot
    to psi_d lists (4 B each) and, with the forward store, copies the pairs
    there (8 B each), 20 psi_d + 8m. Delete reads the psi_d stored coordinates
    (4 B each) and removes the slot from psi_d lists (4 B each), 8 psi_d; the
    column stays as it is."""
    nnz = np.diff(w.docs.indptr)
    two_m = 2 * w.m
    res = {}

    def line(tag, ms, docs, nbytes, full=None):
        r = {"docs": int(docs), "kernel_ms": round(ms, 3), "docs_per_s": round(docs / (ms / 1000.0), 1),
             "alg_GBps": round(nbytes / (ms / 1000.0) / 1e9, 1),
             "hbm_frac": round(nbytes / (ms / 1000.0) / 1e9 / HBM_PEAK_GBS, 4)}
        if full is not None:
            r["alg_GBps_full"] = round(full / (ms / 1000.0) / 1e9, 1)
        log("%-14s %8d docs  %8.3f ms  %12.0f docs/s  alg %7.1f GB/s (%.1f%% of HBM peak)%s" % (
            tag, docs, ms, r["docs_per_s"], r["alg_GBps"], 100 * r["hbm_frac"],
            "" if full is None else "; %.1f GB/s counted in full" % r["alg_GBps_full"]))
        return r

    ins_bytes = lambda psi: float(np.sum(8 * psi + 4 * two_m))
    ins_full = lambda psi: float(np.sum(8 * psi + 4 * two_m + 4 * psi + 8 * psi))
    res["insert_build"] = line("insert build", build["insert_ms"], build["insert_docs"], ins_bytes(nnz),
                               ins_full(nnz))
    if n_upd > 0:
        n_upd = min(n_upd, w.docs.rows)
        ids = np.arange(n_upd, dtype=np.uint32)
        sub = w.docs.take(range(n_upd))
        ix.profile(True)
        ix.delete_batch(ids)
        P.load_docs(ix, sub, ids=ids, compact=False)
        u = ix.profile_read_updates()
        ix.profile(False)
        psi = nnz[:n_upd]
        res["delete"] = line("delete", u["delete_ms"], u["delete_docs"], float(np.sum(8 * psi)))
        res["insert_reuse"] = line("insert reuse", u["insert_ms"], u["insert_docs"], ins_bytes(psi), ins_full(psi))
    res["bytes_per_doc"] = ("insert 8 psi_d + 8m (in full, with list appends and the forward store, "
                            "20 psi_d + 8m); delete 8 psi_d")
    return res


def measured_copy_gbps(torch, dev, mib=1024, reps=10):
    """Achievable HBM bandwidth: a 1 GiB device-to-device copy (bytes read +
    bytes written per second), best of `reps` after one warm-up, on the current
    stream."""
    n = (mib << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = float("inf")
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        best = min(best, a.elapsed_time(b))
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * (mib << 20) / (best / 1000.0) / 1e9


def tile_kernel_name(sched, form):
    """The scoring kernel a form launches under a schedule, as the profiler names
    it (template arguments: slots per lane, bfloat16 sketch, queries per group)."""
    if form == "plain":
        return "k_tiles<%d>" % sched["R_plain"]
    R, Q = sched["R_batch"], sched["qgroup"]
    if Q > 1:
        return ("k_tiles_persistent_grouped<%d, false, %d>" if sched["persistent"] else
                "k_tiles_grouped<%d, false, %d>") % (R, Q)
    return ("k_tiles_persistent<%d>" if sched["persistent"] else "k_tiles<%d>") % R


def kernel_source_sha256():
    """Fingerprint of the scoring kernel's sources (kernels_search.hip and
    snn_device.h) with comments and blank lines left out, so that a comment
    edit does not orphan the counters taken for the same code."""
    import hashlib
    import re

    h = hashlib.sha256()
    for f in ("paper_2301_10622_amd/csrc/kernels_search.hip", "paper_2301_10622_amd/csrc/snn_device.h"):
        text = open(os.path.join(ROOT, f)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for line in text.splitlines():
            line = line.split("//", 1)[0].rstrip()
            if line:
                h.update(line.encode() + b"\n")
    return h.hexdigest()


def measured_counters(kernel, k):
    """Per-launch figures of the committed rocprofv3 passes for this kernel and
    k (HBM bytes from FETCH_SIZE / WRITE_SIZE calibrated against a plain copy,
    VALU instructions from SQ_INSTS_VALU), or None when the kernel source has
    changed since they were taken."""
    path = os.path.join(ROOT, "profiles", "counters.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(kernel)
    if not rec or kernel_source_sha256() != rec["source_sha256"]:
        return None
    return rec.get("k%d" % k)


def compulsory_bytes(np, w, classes, list_len, buckets, sketch_bytes=4):
    """HBM bytes a batch of the workload must read at least once: the posting
    containers of every distinct query coordinate (a bitmap over the used
    slots, or an array container: its row of block offsets, 2 bytes per
    posting, and per sign the coordinate is queried with the stored bound of
    each posting), every sketch row (bucket, U or L half) a query entry of a
    bitmap coordinate touches, over the used slots, the live bitmap, and 16
    bytes per prepared query entry."""
    used = -(-w.docs.rows // 1024) * 1024
    qc = w.queries.coords.astype(np.int64)
    neg = (w.queries.vals < 0).astype(np.int64)
    j = np.unique(qc)
    arr = classes[j] != 0
    cont = float(np.sum(np.where(arr, 2 * list_len[j] + (used // 1024 + 1) * 4, used // 8)))
    signed = np.unique(qc * 2 + neg) // 2  # one per (coordinate, sign) queried
    cont += float(np.sum(np.where(classes[signed] != 0, sketch_bytes * list_len[signed], 0)))
    bm = classes[qc] == 0
    rows = np.unique(np.concatenate([buckets[o][qc[bm]].astype(np.int64) * 2 + neg[bm] for o in range(len(buckets))]))
    return cont + float(len(rows)) * used * sketch_bytes + used / 8 + 16.0 * len(qc)


def oracle_qps(ora, queries, k, threads, reps=3):
    """The FP64 oracle's search rate (Alg. 6 + FindLargest) on `queries`:
    median of `reps` runs on `threads` host threads."""
    import numpy as np

    runs = []
    for _ in range(reps):
        t = time.perf_counter()
        ora.search(queries, k, threads=threads)
        runs.append(time.perf_counter() - t)
    return {"qps": round(queries.rows / float(np.median(runs)), 2), "queries": int(queries.rows), "k": k,
            "threads": threads, "runs_s": [round(x, 3) for x in runs]}


def recall_vs_exact(ora, queries, ids, cnt, k, threads):
    """Mean recall@k of the GPU results (ids, counts: numpy rows of `queries`)
    against the oracle's exact brute-force top-k (Eq. 2)."""
    import numpy as np

    eids, _, _, ecnt = ora.search(queries, k, exact=True, threads=threads)
    r = [len(set(ids[i][: cnt[i]].tolist()) & set(eids[i][: ecnt[i]].tolist())) / max(1, min(k, ecnt[i]))
         for i in range(queries.rows)]
    return float(np.mean(r))


def _rounded(d):
    return {k: (round(v, 4) if isinstance(v, float) else v) for k, v in d.items()}


def batch_4m(args, dev, P, gen, np, torch):
    """Batching workload: 4M docs with the small-index laws, 8,192 queries of nnz
    log-uniform 5..400 in one persistent launch per batch, k = 100."""
    t = time.time()
    w = gen.make_batch(0)
    log("batch4m: generated %d docs / %d queries in %.1fs" % (w.docs.rows, w.queries.rows, time.time() - t))
    ix = P.Index(w.n, w.m, w.h, capacity=w.docs.rows, hash_seed=w.hash_seed, stream=torch.cuda.current_stream())
    P.load_docs(ix, w.docs, compact=not args.no_compact)
    up = lambda q: (torch.tensor(q.indptr, dtype=torch.int64, device=dev),
                    torch.tensor(q.coords.astype(np.int32), device=dev), torch.tensor(q.vals, device=dev))
    et = up(w.queries)
    nq, k = w.queries.rows, 100
    list_len = np.bincount(w.docs.coords, minlength=w.n).astype(np.int64)
    post = np.add.reduceat(list_len[w.queries.coords], w.queries.indptr[:-1])
    ab = float((post * 8 + 12 * np.diff(w.queries.indptr) + 8 * k).sum())
    sched = ix.autotune(*et, k)
    res = {"workload": w.name, "docs": w.docs.rows, "queries_per_step": nq, "k": k, "schedule": sched,
           "alg_bytes_per_step": ab}
    out = (torch.empty((nq, k), dtype=torch.int32, device=dev), torch.empty((nq, k), dtype=torch.float32, device=dev),
           torch.empty(nq, dtype=torch.int32, device=dev))
    for name, mode, steps in (("plain", P.MODE_PLAIN, 1), ("batched", P.MODE_BATCHED, 5)):
        ix.search_batch_dev(*et, k, mode=mode, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ix.search_batch_dev(*et, k, mode=mode, out=out)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1000 / steps
        res[name] = {"qps": round(nq / (ms / 1000), 1), "ms_per_step": round(ms, 3),
                     "alg_GBps": round(ab / (ms / 1000) / 1e9, 1)}
        log("batch4m %-8s %9.3f ms/step %10.0f q/s alg %.0f GB/s" % (name, ms, nq / (ms / 1000), ab / (ms / 1000) / 1e9))
    res["batched_over_plain"] = round(res["batched"]["qps"] / res["plain"]["qps"], 2)
    ix.close()
    # recall@100 against exact brute force on a seeded sample of the batch
    # (plain and batched return identical results)
    from oracle import oracle as O

    S = 64
    rows = np.sort(np.random.default_rng(5).choice(nq, S, replace=False))
    ora = O.Index(w.docs, w.n, w.m, w.h, w.hash_seed)
    g_ids = out[0].cpu().numpy().astype(np.int64)[rows]
    g_cnt = out[2].cpu().numpy()[rows]
    rec = round(recall_vs_exact(ora, w.queries.take(rows), g_ids, g_cnt, k, O.max_threads()), 4)
    for name in ("plain", "batched"):
        res[name]["recall_at_100"] = rec
    res["recall_sample"] = "%d seeded queries of the batch" % S
    log("batch4m recall@100 %.4f (%d queries)" % (rec, S))
    if not args.no_cpu_baseline:
        sub = w.queries.take(np.sort(np.random.default_rng(6).choice(nq, 512, replace=False)))
        res["cpu_oracle"] = oracle_qps(ora, sub, k, O.max_threads())
        res["cpu_oracle"]["sample"] = "512 seeded queries of the batch"
        log("batch4m oracle %.1f q/s (512 queries)" % res["cpu_oracle"]["qps"])
    del ora
    return res


def paper_gaussian(args, dev, P, gen, np, torch, psi):
    """The real-valued collections of Section 6.5 (Table 4): 5M docs, every
    coordinate non-zero with probability psi / n, N(0, 1) values; k = 1,000 and
    k' = 20,000, 2m = 74 (G100) or 150 (G200), h = 1, as the paper runs them. The
    anytime budget is a count of coordinates here (the paper's T is in ms).
    1,000 queries in batches of 200; recall@1000 against exact brute force and
    agreement with the oracle's Alg. 7 on a query sample."""
    from oracle import oracle as O

    t = time.time()
    w = gen.make_gaussian(0, psi)
    log("g%d: generated %d docs (nnz %d) / %d queries in %.1fs" % (psi, w.docs.rows, w.docs.nnz, w.queries.rows,
                                                                    time.time() - t))
    stream = torch.cuda.current_stream()
    ix = P.Index(w.n, w.m, w.h, capacity=w.docs.rows, hash_seed=w.hash_seed, stream=stream, forward_store=True)
    t = time.time()
    P.load_docs(ix, w.docs, compact=not args.no_compact)
    torch.cuda.synchronize()
    t_ins = time.time() - t
    k, kp, B = 1000, 20000, 200
    nq = w.queries.rows
    batches = []
    for b0 in range(0, nq, B):
        q = w.queries.take(range(b0, min(nq, b0 + B)))
        batches.append((torch.tensor(q.indptr, dtype=torch.int64, device=dev),
                        torch.tensor(q.coords.astype(np.int32), device=dev), torch.tensor(q.vals, device=dev),
                        q.rows))
    res = {"workload": w.name, "docs": w.docs.rows, "dim": w.n, "m": w.m, "queries": nq, "k": k, "k_prime": kp,
           "insert_docs_per_s_host_api": round(w.docs.rows / t_ins, 1), "forms": {}}
    # the batched schedule, tuned on the first batch at k = 1,000
    ip0, qc0, qv0, _ = batches[0]
    if args.schedule:
        R, Q, grid, pers = [int(x) for x in args.schedule.split(",")]
        ix.set_schedule(16, R, grid, bool(pers), Q)
        res["schedule"] = ix.schedule()
    else:
        res["schedule"] = ix.autotune(ip0, qc0, qv0, k, total=int(qc0.numel()))
    log("g%d: schedule %s" % (psi, res["schedule"]))
    outs = {}
    budgets = (0, 50, 25) if psi == 100 else (0, 100, 50)
    for c in budgets:
        out = [(torch.empty((nb, k), dtype=torch.int32, device=dev), torch.empty((nb, k), dtype=torch.float32,
                                                                                 device=dev),
                torch.empty(nb, dtype=torch.int32, device=dev)) for (_, _, _, nb) in batches]

        def run_all():
            for (ip, qc, qv, nb), o in zip(batches, out):
                ix.search_ex_dev(ip, qc, qv, k, k_prime=kp, max_coords=c, out=o)

        run_all()  # warm-up (captures the graphs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = 2
        for _ in range(reps):
            run_all()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1000 / reps
        outs[c] = out
        # one query alone: latency
        ip1 = torch.tensor(w.queries.indptr[:2], dtype=torch.int64, device=dev)
        qc1 = batches[0][1][: int(w.queries.indptr[1])].contiguous()
        qv1 = batches[0][2][: int(w.queries.indptr[1])].contiguous()
        o1 = (torch.empty((1, k), dtype=torch.int32, device=dev), torch.empty((1, k), dtype=torch.float32, device=dev),
              torch.empty(1, dtype=torch.int32, device=dev))
        ix.search_ex_dev(ip1, qc1, qv1, k, k_prime=kp, max_coords=c, out=o1)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(5):
            ix.search_ex_dev(ip1, qc1, qv1, k, k_prime=kp, max_coords=c, out=o1)
        torch.cuda.synchronize()
        lat = (time.perf_counter() - t1) * 1000 / 5
        name = "coords=%s" % (c or "all")
        res["forms"][name] = {"qps": round(nq / (ms / 1000), 1), "ms_per_1000_queries": round(ms, 2),
                              "single_query_ms": round(lat, 3)}
        log("g%d %-12s %9.2f ms / %d queries  %9.0f q/s  one query alone %.2f ms" % (psi, name, ms, nq,
                                                                                     nq / (ms / 1000), lat))
    # recall and agreement with the oracle on a sample
    S = 8
    log("g%d: building the FP64 oracle" % psi)
    t = time.time()
    ora = O.Index(w.docs, w.n, w.m, w.h, w.hash_seed)
    log("g%d: oracle index %.1fs" % (psi, time.time() - t))
    sample = w.queries.take(range(S))
    eids, _, _, ecnt = ora.search(sample, k, exact=True, threads=O.max_threads())
    for c in budgets:
        rids, _, _, rcnt = ora.rerank(sample, k, kp, threads=O.max_threads(), max_coords=c)
        g_ids = outs[c][0][0][:S].cpu().numpy().astype(np.int64)
        g_cnt = outs[c][0][2][:S].cpu().numpy()
        rec = [len(set(g_ids[i][: g_cnt[i]].tolist()) & set(eids[i][: ecnt[i]].tolist())) / k for i in range(S)]
        same = [len(set(g_ids[i][: g_cnt[i]].tolist()) & set(rids[i][: rcnt[i]].tolist())) / k for i in range(S)]
        name = "coords=%s" % (c or "all")
        res["forms"][name]["recall_at_%d" % k] = round(float(np.mean(rec)), 4)
        res["forms"][name]["overlap_with_oracle_alg7"] = round(float(np.mean(same)), 4)
        log("g%d %s: recall@%d %.4f, id overlap with the oracle's Alg. 7 %.4f (%d queries)" % (
            psi, name, k, np.mean(rec), np.mean(same), S))
    res["paper_table4_context"] = ("CPU (the paper's Intel setup), Sinnamon 2m=%d: T=40 ms -> %s, T=20 ms -> %s" %
                                   ((74, "87 ms, recall 0.97", "66 ms, recall 0.89") if psi == 100 else
                                    (150, "107 ms, recall 0.92", "86 ms, recall 0.83")))
    del ora
    ix.close()
    return res


def serving_8m(args, dev, P, gen, np, torch):
    """Serving workload: capacity 8M slots, 4M prefilled small-law docs; Poisson
    arrivals of 85% searches (nnz lognormal mean 40, k in {10, 100, 1000}), 10%
    inserts, 5% deletes; admission by a device-memory budget; p50 / p99."""
    t = time.time()
    docs = gen.small_docs(0, 4_000_000)
    log("serving: generated prefill in %.1fs" % (time.time() - t))
    ix = P.Index(1000, 32, 1, capacity=8_000_000, hash_seed=0, stream=torch.cuda.current_stream())
    P.load_docs(ix, docs, compact=not args.no_compact)
    ops = args.serving_ops
    res = {"workload": "serving capacity 8M, 4M prefill, %d ops, 85/10/5 search/insert/delete" % ops}
    # the batched schedule, tuned on 1,024 queries of the serving law at k = 100
    sq = gen.serving_queries(7, 1024)
    et = (torch.tensor(sq.indptr, dtype=torch.int64, device=dev), torch.tensor(sq.coords.astype(np.int32), device=dev),
          torch.tensor(sq.vals, device=dev))
    res["schedule"] = ix.autotune(*et, 100, total=int(sq.nnz))
    del et
    log("serving: schedule %s" % res["schedule"])
    budget = 8 << 30
    # recall@k of the serving index against exact brute force, on the
    # prefilled state, for 64 queries of the serving law at each k of the mix
    from oracle import oracle as O

    rq = gen.serving_queries(9, 64)
    ora = O.Index(docs, 1000, 32, 1, 0)
    res["recall_prefill"] = {}
    for kk in (10, 100, 1000):
        g_ids, _, g_cnt = ix.search_batch(rq.indptr, rq.coords, rq.vals, kk)
        res["recall_prefill"]["recall_at_%d" % kk] = round(
            recall_vs_exact(ora, rq, g_ids.astype(np.int64), g_cnt, kk, O.max_threads()), 4)
    if not args.no_cpu_baseline:
        res["cpu_oracle"] = oracle_qps(ora, gen.serving_queries(10, 512), 100, O.max_threads())
        res["cpu_oracle"]["sample"] = "512 queries of the serving law on the prefilled index, k = 100"
        log("serving oracle %.1f q/s (512 queries)" % res["cpu_oracle"]["qps"])
    del ora
    log("serving recall on the prefilled index (64 queries): %s" % res["recall_prefill"])

    live = {"ids": np.arange(docs.rows, dtype=np.int64)}

    def run(rate, realtime, seed):
        tr = gen.serving_trace(seed, ops, live["ids"], 10_000_000 + seed * 1_000_000, rate)
        csr = gen.trace_csr(tr)
        # the live set after this trace (the next trace deletes from it)
        gone = set(tr["ids"][tr["kind"] == 2].tolist())
        keep = live["ids"][~np.isin(live["ids"], list(gone))] if gone else live["ids"]
        live["ids"] = np.concatenate([keep, tr["ids"][tr["kind"] == 1].astype(np.int64)])
        _, _, cnt, lat, rep = ix.serve(tr["kind"], tr["t"], tr["ids"], tr["k"], csr.indptr, csr.coords, csr.vals,
                                       max_batch=1024, max_inflight=3, streams=3, realtime=realtime,
                                       budget_bytes=budget)
        return _rounded(rep)

    sat = run(1e9, False, 1)
    res["saturated"] = sat
    log("serving saturated: %.0f q/s (batches %d, max in flight %d)" % (
        sat["search_qps"], sat["batches"], sat["max_inflight_seen"]))
    for frac, seed in ((0.5, 2), (0.8, 3), (0.95, 4)):
        rep = run(sat["search_qps"] * frac, True, seed)
        res["load_%.2f" % frac] = rep
        log("serving at %.2f x saturation: %.0f q/s  p50 %.3f ms  p99 %.3f ms  mutations p99 %.3f ms" % (
            frac, rep["search_qps"], rep["p50_ms"], rep["p99_ms"], rep["mutation_p99_ms"]))
    res["budget_bytes"] = budget
    ix.close()
    return res


def small_learned(args, dev, P, gen, np, torch):
    """The learned-filter workload: the 10k-doc index, 200,000 training queries
    labelled by the plain method, 8,192 evaluation queries, k = 10."""
    w = gen.make_small(0)
    ix = P.Index(w.n, w.m, w.h, capacity=w.docs.rows, hash_seed=w.hash_seed, stream=torch.cuda.current_stream())
    P.load_docs(ix, w.docs, compact=not args.no_compact)
    tq = gen.small_queries(2, 200_000)
    eq = gen.small_queries(3, 8192)
    up = lambda q: (torch.tensor(q.indptr, dtype=torch.int64, device=dev),
                    torch.tensor(q.coords.astype(np.int32), device=dev), torch.tensor(q.vals, device=dev))
    tt, et = up(tq), up(eq)
    sched = ix.autotune(*et, 10)
    rep = ix.filter_train(*tt, k=10, epochs=8, batch=1024, lr=1e-3, target_fallback=args.filter_fallback)
    log("small: filter trained: %s" % rep)
    nq = eq.rows
    out = (torch.empty((nq, 10), dtype=torch.int32, device=dev), torch.empty((nq, 10), dtype=torch.float32, device=dev),
           torch.empty(nq, dtype=torch.int32, device=dev))
    res = {"workload": "small-10k-dim1000 learned filter, 8192 eval queries, k=10", "schedule": sched,
           "filter": {kk: (round(v, 4) if isinstance(v, float) else v) for kk, v in rep.items()}}
    ref = None
    for name, mode, steps in (("plain", P.MODE_PLAIN, 2), ("batched", P.MODE_BATCHED, 20), ("learned", P.MODE_LEARNED, 20)):
        ix.search_batch_dev(*et, 10, mode=mode, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ix.search_batch_dev(*et, 10, mode=mode, out=out)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1000 / steps
        got = [x.cpu().numpy().copy() for x in out]
        if ref is None:
            ref = got
        same = all(np.array_equal(a, b) for a, b in zip(ref, got))
        res[name] = {"qps": round(nq / (ms / 1000), 1), "ms_per_step": round(ms, 4), "identical_to_plain": same}
        if name == "learned":
            res[name]["fallbacks"] = ix.last_batch_status()[1]
        log("small %-8s %8.3f ms/step %10.0f q/s identical=%s" % (name, ms, nq / (ms / 1000), same))
    res["learned_over_batched"] = round(res["learned"]["qps"] / res["batched"]["qps"], 3)
    res["learned_over_plain"] = round(res["learned"]["qps"] / res["plain"]["qps"], 3)
    ix.close()
    # recall@10 against exact brute force over every evaluation query (the
    # three forms return identical results)
    from oracle import oracle as O

    ora = O.Index(w.docs, w.n, w.m, w.h, w.hash_seed)
    rec = round(recall_vs_exact(ora, eq, ref[0].astype(np.int64), ref[2], 10, O.max_threads()), 4)
    for name in ("plain", "batched", "learned"):
        res[name]["recall_at_10"] = rec
    log("small recall@10 %.4f (%d queries)" % (rec, nq))
    if not args.no_cpu_baseline:
        res["cpu_oracle"] = {"small_100_queries": oracle_qps(ora, w.queries, 10, O.max_threads()),
                             "eval_queries": oracle_qps(ora, eq, 10, O.max_threads())}
        log("small oracle %.1f q/s (100 queries), %.1f q/s (%d evaluation queries)" % (
            res["cpu_oracle"]["small_100_queries"]["qps"], res["cpu_oracle"]["eval_queries"]["qps"], nq))
    return res


if __name__ == "__main__":
    main()
