"""Benchmark: encrypted 128x128x128 matrix product with unstructured sparsity.

One step = one encrypted C = A*B (N = 2^14; five data primes of 60/40/40/40/40
bits and three 60-bit special primes; hybrid key switching with dnum = 2;
scale 2^40) with A 128x128 at 50% unstructured sparsity in CSR and B 128x128
dense: every nonzero ciphertext product (tensor), one key switch and one
rescale per output (the lazy, batched form).  Inputs are encrypted and
resident in HBM before the timed region; setup, key generation, encryption and
decryption are excluded, as in the paper's profiling procedure (Sec. 4.1).

Prints one JSON line.  `value` is ct-mults/s: executed ciphertext products
per second of the headline step.  Beside it: the same at 90% sparsity, the
naive dense schedule on the same operands, the per-product (Algorithm 1 order)
form, the other two sparse encodings, the dominant kernel's roofline, and the
CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np

# MI355X published peaks
HBM_PEAK_GBS = 8000.0
# VALU lane-op peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3 T lane-op/s,
# the issue rate of full-rate VALU instructions (fp64 FMA/MUL/RNDNE,
# v_mad_u64_u32), i.e. the published 78.6 TFLOP/s fp64 vector peak / 2.
VALU_PEAK = 256 * 4 * 16 * 2.4e9
# Algorithmic VALU ops per ciphertext product per prime and coefficient in the
# fp64 residue arithmetic (primes below 2^42): three exact products
# a*b - rint(a*b/q)*q (mul, fma, mul, rndne, fma, add) for a0 b0, a1 b1 and
# the Karatsuba (a0+a1)(b0+b1), plus three accumulating adds.
FP_OPS_PER_PRODUCT = 21
# ... in the carry-save arithmetic of the primes 2^60 - c (c < 2^20): 16
# v_mad_u64_u32 (four 30-bit partial products for each of a0 b0, a0 b1,
# a1 b0, a1 b1), the fold every four entries not counted
INT60_OPS_PER_PRODUCT = 16
# Fused key switch + rescale of one output at N = 2^14 with five data and
# three special primes (dnum = 2): 32 transforms of 2^13 * 14 = 114,688
# butterflies each, 16 of them over the 60-bit primes (integer Harvey
# butterflies with Shoup twiddles: about 28 VALU instructions each) and 16
# over the 40-bit primes (exact fp64 butterflies: 8 each); the base
# conversions and key products (about 90 modular products per coefficient)
# are HBM-bound element-wise work and are not counted here.
KS_BUTTERFLIES_PER_TRANSFORM = (1 << 13) * 14
KS_INT_TRANSFORMS, KS_FP_TRANSFORMS = 16, 16
KS_INT_OPS_PER_BUTTERFLY, KS_FP_OPS_PER_BUTTERFLY = 28, 8
KS_OPS_PER_OUTPUT = KS_BUTTERFLIES_PER_TRANSFORM * (KS_INT_TRANSFORMS * KS_INT_OPS_PER_BUTTERFLY +
                                                    KS_FP_TRANSFORMS * KS_FP_OPS_PER_BUTTERFLY)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "tensor_fp_traffic.json")


def source_digest():
    import hashlib
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_2503_09184_amd", "csrc", "tensor.hip"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the fp64 tensor kernel from the committed
    rocprofv3 FETCH_SIZE/WRITE_SIZE measurement, if it was taken on this
    kernel source (else None)."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("tensor_hip_sha256_16") != source_digest():
        return None
    return t.get("bytes_per_launch")


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def measured_peaks(torch, sfhe):
    """What this chip sustains: a 1 GiB device copy (bytes read + written per
    second) and the VALU issue-rate probes of the library."""
    n_words = (1 << 30) // 8
    src = torch.ones(n_words, dtype=torch.int64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 5 * 2 * (1 << 30) / (e0.elapsed_time(e1) / 1e3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    out = {"copy_GBps": copy_gbs}
    for kind in ("fp64_fma", "mad_u64_u32", "int32_add"):
        out[kind + "_Tops"] = sfhe.probe_valu(kind) / 1e12
    return out


def summary(times):
    return {"mean": float(np.mean(times)), "median": float(np.median(times)), "min": float(np.min(times)),
            "max": float(np.max(times)), "n": len(times)}


def step_ops(products, keyswitches, N, n_fp, n_int60):
    """Algorithmic VALU operations of one product step at N = 2^14 with the
    benchmarked primes: the tensor products (21 per product, prime and
    coefficient in fp64, 16 in the carry-save integer arithmetic) and the
    transforms of the fused key switch and rescale per output."""
    return (float(products) * N * (n_fp * FP_OPS_PER_PRODUCT + n_int60 * INT60_OPS_PER_PRODUCT) +
            float(keyswitches) * KS_OPS_PER_OUTPUT)


def timed(ctx, torch, A, B, sched, steps, warmup, keep_last=False):
    """Run warmup + steps matmuls; return (ms per step list, stats of the last,
    last C or None, [(fp64 tensor kernel ms, launches)] per timed step)."""
    stream = torch.cuda.current_stream()
    C = None
    for _ in range(warmup):
        C = ctx.matmul(A, B, sched)
        C.close()
    torch.cuda.synchronize()
    times = []
    stats = None
    fp = []   # (fp64 tensor kernel ms, its launches) of every timed step
    for s in range(steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        C = ctx.matmul(A, B, sched)
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
        stats = ctx.last_stats()
        fp.append((stats.tensor_fp_ms, int(stats.tensor_fp_launches)))
        if not (keep_last and s == steps - 1):
            C.close()
            C = None
    return times, stats, C, fp


def cpu_baseline(P, A, Bm, seed, threads, target_s=15.0):
    """The oracle on a bounded sample of outputs of the same workload (lazy, CSR).

    The oracle assigns output (i, j) to thread (i*cols + j) mod T, so a sample
    of every row times a multiple of T columns keeps the threads balanced."""
    from oracle.oracle import Oracle
    from paper_2503_09184_amd import workloads as W
    orc = Oracle(**P)
    orc.keygen(W.key_seed(seed))
    sa, sb = W.enc_seed(seed, 0), W.enc_seed(seed, 1)
    M, Nc = A.shape[0], Bm.shape[1]
    probe = [(0, j) for j in range(threads)]
    _, _, t_probe = orc.matmul(A, Bm, "csr", "lazy", sa, sb, outputs=probe, threads=threads, decrypt=False)
    per_output_thread = max(t_probe, 1e-4)            # one output per thread
    want_outputs = target_s / per_output_thread * threads
    cols = int(min(Nc, max(threads, round(want_outputs / M / threads) * threads)))
    outs = [(i, j) for i in range(M) for j in range(cols)]
    _, _, secs = orc.matmul(A, Bm, "csr", "lazy", sa, sb, outputs=outs, threads=threads, decrypt=False)
    products = sum(int(np.count_nonzero(A[i])) for (i, _) in outs)
    return {"value": products / secs, "unit": "ct-mults/s", "cores": threads, "kind": "oracle",
            "sample": "%d outputs (all %d rows x columns 0-%d) of the 50%%-sparse CSR lazy product: %d ct "
                      "products, %.1f s on %d threads" % (len(outs), M, cols - 1, products, secs, threads),
            "seconds": secs, "products": products}


# plaintext weights times encrypted values: one output's sum (five primes,
# two polys) and its rescaled result (four primes), and one stored ciphertext
PLAIN_SUM_MIB, PLAIN_OUT_MIB, PLAIN_CT_MIB = 1.25, 1.0, 1.25


def ctpt_leg(torch, sfhe, W, count=32):
    """The uneven batch of plaintext-weight products: count independent W B
    with M, K, Nc drawn from {32, 64, 128, 256} and W's zero fraction uniform
    on [0.5, 0.9], N = 2^14, B encrypted per element.  The whole batch does not
    fit in HBM at once (about 1.4 TB of operands, sums and results), so it runs
    in waves admitted by memory: a job whose operands, sums and results exceed
    the wave budget is split into column blocks of B, and each wave is one
    fused batch call.  Encryption and encoding are outside the timed calls.
    The one-launch-per-product form is timed on the job with the fewest
    products, beside the fused form on that job, and both again captured into
    a HIP graph and replayed."""
    P = W.PARAMS["plain_n16384"]
    cfg = 4
    ctx = sfhe.Context(**P)
    ctx.keygen(W.key_seed(cfg))
    jobs = W.uneven_batch(W.workload_seed(cfg), count)
    free, _ = torch.cuda.mem_get_info()
    budget_mib = min(0.45 * free / 2 ** 20, 120 * 1024.0)
    units = []   # (job, M, K, col0, ncols, sparsity)
    for jn, (M, K, Nc, s) in enumerate(jobs):
        per_col = K * PLAIN_CT_MIB + M * (PLAIN_SUM_MIB + PLAIN_OUT_MIB)
        blk = max(1, min(Nc, int(budget_mib // per_col)))
        for c0 in range(0, Nc, blk):
            units.append((jn, M, K, c0, min(blk, Nc - c0), s))
    waves, cur, used = [], [], 0.0
    for u in units:
        need = u[4] * (u[2] * PLAIN_CT_MIB + u[1] * (PLAIN_SUM_MIB + PLAIN_OUT_MIB))
        if cur and used + need > budget_mib:
            waves.append(cur)
            cur, used = [], 0.0
        cur.append(u)
        used += need
    if cur:
        waves.append(cur)
    ops = {jn: W.operands(M, K, Nc, s, W.workload_seed(cfg) + 1 + jn) for jn, (M, K, Nc, s) in enumerate(jobs)}
    total_ms, products, launches, wall = 0.0, 0, 0, 0.0
    for wn, wave in enumerate(waves):
        Ws = [ctx.encode_weights(ops[jn][0], "csr", 40) for (jn, M, K, c0, nc, s) in wave]
        Bs = [ctx.encrypt(ops[jn][1][:, c0:c0 + nc], "dense", W.enc_seed(cfg, 1) + jn, 1)
              for (jn, M, K, c0, nc, s) in wave]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Cs = ctx.matmul_plain_batch(Ws, Bs, "fused")
        st = ctx.last_stats()
        wall += time.perf_counter() - t0
        total_ms += st.ms
        products += st.products
        launches += st.tensor_launches
        log("ctpt wave %d/%d: %d products in %d units, %.1f ms" % (wn + 1, len(waves), st.products, len(wave), st.ms))
        for x in Cs + Bs + Ws:
            x.close()
        del Cs, Bs, Ws
    ctx.close()
    torch.cuda.empty_cache()
    return {"matmuls": len(jobs), "shapes_MKN_sparsity": [list(j) for j in jobs], "waves": len(waves),
            "units": len(units), "products": int(products), "ms": total_ms,
            "ctpt_mults_per_s": products / (total_ms / 1e3), "fused_launches": int(launches),
            "host_wall_s": wall}


def ctpt_launch_leg(torch, sfhe, W, count=32):
    """The one-launch-per-product form of the plaintext-weight product against
    the fused form, on the job of the uneven batch (the ct_pt leg's jobs) with
    the fewest products, each also captured into a HIP graph and replayed."""
    P = W.PARAMS["plain_n16384"]
    cfg = 4
    ctx = sfhe.Context(**P)
    ctx.keygen(W.key_seed(cfg))
    jobs = W.uneven_batch(W.workload_seed(cfg), count)
    ops = {jn: W.operands(M, K, Nc, s, W.workload_seed(cfg) + 1 + jn) for jn, (M, K, Nc, s) in enumerate(jobs)}
    jn = min(range(len(jobs)), key=lambda x: int(np.count_nonzero(ops[x][0])) * jobs[x][2])
    Wm = ctx.encode_weights(ops[jn][0], "csr", 40)
    Bm = ctx.encrypt(ops[jn][1], "dense", W.enc_seed(cfg, 1) + jn, 1)
    sample = {"job": list(jobs[jn][:3]), "sparsity": jobs[jn][3]}
    for mode in ("fused", "per_product"):
        ctx.matmul_plain_batch([Wm], [Bm], mode)[0].close()   # warm-up
        C = ctx.matmul_plain_batch([Wm], [Bm], mode)[0]
        stx = ctx.last_stats()
        C.close()
        sample[mode + "_ms"] = stx.ms
        sample["products"] = int(stx.products)
        sample[mode + "_launches"] = int(stx.tensor_launches)
    # the same launches captured into a HIP graph and replayed
    for mode in ("fused", "per_product"):
        g = sfhe.PlainGraph(ctx, [Wm], [Bm], mode)
        g.launch()
        g.launch()
        sample["graph_" + mode + "_ms"] = ctx.last_stats().ms
        g.close()
    sample["fused_over_per_product"] = sample["per_product_ms"] / sample["fused_ms"]
    sample["graph_fused_over_graph_per_product"] = sample["graph_per_product_ms"] / sample["graph_fused_ms"]
    log("ctpt per-product launches on %s: %.2f ms vs fused %.2f ms; as graphs %.2f vs %.2f ms" %
        (sample["job"], sample["per_product_ms"], sample["fused_ms"], sample["graph_per_product_ms"],
         sample["graph_fused_ms"]))
    Wm.close()
    Bm.close()
    ctx.close()
    torch.cuda.empty_cache()
    return sample


def slots_leg(ctx, torch, A, Bm, sa, sb, chunk, sched="lazy"):
    """Algorithm 1 with chunks of `chunk` values per ciphertext (rotations into
    slot 0, the slot-0 mask, rotation to the output slot) on the given
    operands: one untimed call (it builds the rotation keys), then one timed
    call."""
    EA = ctx.encrypt_slots(A, "csr", chunk, sa, 0)
    EB = ctx.encrypt_slots(Bm, "dense", chunk, sb, 1)
    torch.cuda.synchronize()
    ctx.matmul_slots(EA, EB, sched).close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    C = ctx.matmul_slots(EA, EB, sched)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3
    st = ctx.last_stats()
    err = float(np.max(np.abs(ctx.decrypt(C) - A @ Bm)))
    out = {"ms": st.ms, "wall_ms": wall, "products": int(st.products), "ct_mults_per_s": st.products / (st.ms / 1e3),
           "keyswitches_and_rotations": int(st.keyswitches), "chunk": chunk,
           "ciphertexts_A": int(EA.info().n_ciphertexts), "ciphertexts_B": int(EB.info().n_ciphertexts),
           "ciphertexts_C": int(C.info().n_ciphertexts), "max_abs_err_vs_fp64": err}
    for M in (C, EA, EB):
        M.close()
    torch.cuda.empty_cache()
    return out


# (name, server streams, running batches per stream (0: no limit), batch
# byte limit as a fraction of the budget (0: none))
SERVING_POLICIES = [("fifo_1_stream", 1, 0, 0.0), ("2_streams", 2, 0, 0.0), ("2_streams_1_slot_each", 2, 1, 0.0),
                    ("2_streams_half_budget_batches", 2, 0, 0.5)]


def serving_leg(torch, sfhe, W, n_requests=96, load=0.8, pool_per_layer=2):
    """The request loop over plaintext-weight products: encrypted MLP-layer
    requests (weights 128x784, 256x256 or 128x512, i.e. layers 784->128,
    256->256, 512->128, at 50, 75 or 90% zeros; activation batches of 1-16
    columns) arriving as a Poisson process, admitted by memory and batched by
    sfhe_server_step as they arrive.  The layers' weights are encoded once;
    the encrypted activations come from a pool of pool_per_layer matrices per
    layer, encrypted before the run (the client's side; requests only read
    them).  The arrival rate is `load` times the service rate measured on one
    request of each layer alone.  Latency is arrival to result, host clock.
    The same arrivals are served under each admission policy of
    SERVING_POLICIES (server streams, running batches per stream, batch byte
    limit); the first is the reported one."""
    P = W.PARAMS["serving_n32768"]
    cfg = 5
    ctx = sfhe.Context(**P)
    ctx.keygen(W.key_seed(cfg))
    rng = np.random.default_rng(W.workload_seed(cfg))
    layers = [(784, 128), (256, 256), (512, 128)]
    sparsities = [0.5, 0.75, 0.9]
    weights = {}
    for li, (fin, fout) in enumerate(layers):
        for si, sp in enumerate(sparsities):
            Wt = W.sparse_matrix(fout, fin, sp, W.workload_seed(cfg) + 10 * li + si)
            weights[(li, si)] = (Wt, ctx.encode_weights(Wt, "csr", 40))
    pool = {}
    for li in range(3):
        for x in range(pool_per_layer):
            b = int(rng.integers(1, 17))
            X = W.uniform_matrix(layers[li][0], b, W.workload_seed(cfg) + 1000 + 100 * li + x)
            pool[(li, x)] = (b, X, ctx.encrypt(X, "dense", W.enc_seed(cfg, 1) + 100 * li + x, 1))
    reqs = []
    for n in range(n_requests):
        li, si, x = int(rng.integers(3)), int(rng.integers(3)), int(rng.integers(pool_per_layer))
        b, X, EX = pool[(li, x)]
        reqs.append({"layer": li, "sp": si, "b": b, "X": X, "EX": EX})
    torch.cuda.synchronize()
    free, _ = torch.cuda.mem_get_info()
    budget = int(min(0.5 * free, 64 << 30))
    # service time of one request alone, per layer, at 8 columns
    alone_ms = []
    for li in range(3):
        r = next((q for q in reqs if q["layer"] == li), reqs[0])
        srv = sfhe.Server(ctx, budget)
        t = srv.submit(weights[(r["layer"], 1)][1], r["EX"])
        srv.step()
        srv.poll(t, wait=True)[1].close()
        t0 = time.perf_counter()
        t = srv.submit(weights[(r["layer"], 1)][1], r["EX"])
        srv.step()
        srv.poll(t, wait=True)[1].close()
        alone_ms.append((time.perf_counter() - t0) * 1e3 * 8.0 / r["b"])
        srv.close()
    mean_service_s = float(np.mean(alone_ms)) * (8.5 / 8.0) / 1e3
    rate = load / mean_service_s
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=n_requests))
    # a result in the mix is compared with the same request alone, bit for bit
    checked = (0, n_requests // 2, n_requests - 1)
    solo_cts = {}
    for n in checked:
        r = reqs[n]
        solo = sfhe.Server(ctx, budget)
        t = solo.submit(weights[(r["layer"], r["sp"])][1], r["EX"])
        solo.step()
        C1 = solo.poll(t, wait=True)[1]
        solo_cts[n] = [ctx.export_ct(C1, i, j) for (i, j) in [(0, 0), (layers[r["layer"]][1] - 1, r["b"] - 1)]]
        C1.close()
        solo.close()

    def serve(n_streams, slots, cap_frac):
        srv = sfhe.Server(ctx, budget, n_streams=n_streams, slots=slots, batch_bytes=int(budget * cap_frac))
        tickets, done_at, results, sizes = {}, {}, {}, []
        step_s, step_max = 0.0, 0.0
        t0 = time.perf_counter()
        nxt = 0
        while len(done_at) < n_requests:
            now = time.perf_counter() - t0
            while nxt < n_requests and arrivals[nxt] <= now:
                r = reqs[nxt]
                tickets[nxt] = srv.submit(weights[(r["layer"], r["sp"])][1], r["EX"])
                nxt += 1
            ts = time.perf_counter()
            srv.step()
            dt = time.perf_counter() - ts
            step_s += dt
            step_max = max(step_max, dt)
            for n, t in tickets.items():
                if n in done_at:
                    continue
                d, C, ms, bs = srv.poll(t)
                if d:
                    done_at[n] = time.perf_counter() - t0
                    if n in checked:
                        results[n] = C          # kept for the checks below
                    else:
                        C.close()
                    sizes.append(bs)
            if nxt < n_requests and not any(n not in done_at for n in tickets):
                time.sleep(max(0.0, min(arrivals[nxt] - (time.perf_counter() - t0), 0.002)))
            else:
                time.sleep(0.0002)
        makespan = max(done_at.values()) - arrivals[0]
        st = srv.status()
        # batches whose device-time interval intersects another batch's ran concurrently
        iv = sorted(set(srv.intervals[t] for t in tickets.values()))
        overl = sum(1 for x in range(len(iv)) if any(iv[x][0] < iv[y][1] and iv[y][0] < iv[x][1]
                                                   for y in range(len(iv)) if y != x))
        busy = 0.0
        cur0, cur1 = None, None
        for a, b in iv:
            if cur1 is None or a > cur1:
                if cur1 is not None:
                    busy += cur1 - cur0
                cur0, cur1 = a, b
            else:
                cur1 = max(cur1, b)
        if cur1 is not None:
            busy += cur1 - cur0
        lat = np.array([(done_at[n] - arrivals[n]) * 1e3 for n in range(n_requests)])
        same = all(np.array_equal(ctx.export_ct(results[n], i, j), solo_cts[n][x])
                   for n in checked
                   for x, (i, j) in enumerate([(0, 0), (layers[reqs[n]["layer"]][1] - 1, reqs[n]["b"] - 1)]))
        err = max(float(np.max(np.abs(ctx.decrypt(results[n]) -
                                      weights[(reqs[n]["layer"], reqs[n]["sp"])][0] @ reqs[n]["X"])))
                  for n in (0, n_requests - 1))
        for C in results.values():
            C.close()
        srv.close()
        return {"streams": n_streams, "slots_per_stream": slots, "batch_bytes_limit": int(budget * cap_frac),
                "latency_ms_p50": float(np.percentile(lat, 50)), "latency_ms_p99": float(np.percentile(lat, 99)),
                "latency_ms_mean": float(lat.mean()), "makespan_s": makespan, "products": int(st["products"]),
                "ctpt_mults_per_s": st["products"] / makespan, "batches": int(st["batches"]),
                "mean_batch_size": float(np.mean(sizes)), "max_batch_size": int(max(sizes)),
                "alone_equals_mix": bool(same), "max_abs_err_vs_fp64": err,
                "batches_overlapping_another": overl, "device_busy_ms": busy,
                "device_batch_ms_sum": float(sum(b - a for a, b in iv)),
                "host_step_ms_sum": step_s * 1e3, "host_step_ms_max": step_max * 1e3}

    policies = {}
    for name, n_streams, slots, cap_frac in SERVING_POLICIES:
        policies[name] = serve(n_streams, slots, cap_frac)
        log("serving %s: p50 %.1f ms, p99 %.1f ms, %d batches, %d overlapping, host step %.0f ms" %
            (name, policies[name]["latency_ms_p50"], policies[name]["latency_ms_p99"], policies[name]["batches"],
             policies[name]["batches_overlapping_another"], policies[name]["host_step_ms_sum"]))
    for k in pool:
        pool[k][2].close()
    for k in weights:
        weights[k][1].close()
    ctx.close()
    torch.cuda.empty_cache()
    out = {"requests": n_requests, "load": load, "arrival_rate_per_s": rate, "budget_gib": budget / 2 ** 30,
           "policy": SERVING_POLICIES[0][0], "ring": "N=2^15, 9 data + 3 special primes (12 limbs), dnum=3"}
    out.update(policies[SERVING_POLICIES[0][0]])
    out["policies"] = policies
    return out


def cpu_thread_scaling(threads, target_s=8.0):
    """The paper-style thread speed-up (Sec. 4.3) of the oracle on the sweep
    ring (N = 2^13, 64 x 64 x 64, A 50% zeros in CSR, PER_PRODUCT: every
    product relinearised and rescaled, as in the paper): the same sample of
    outputs on one thread and on `threads` threads (output (i, j) on thread
    (i * 64 + j) mod T)."""
    from oracle.oracle import Oracle
    from paper_2503_09184_amd import workloads as W
    P = W.PARAMS["sweep_n8192"]
    orc = Oracle(**P)
    orc.keygen(W.key_seed(2))
    A, B = W.operands(64, 64, 64, 0.5, W.workload_seed(2))
    sa, sb = W.enc_seed(2, 0), W.enc_seed(2, 1)
    _, _, t1 = orc.matmul(A, B, "csr", "per_product", sa, sb, outputs=[(0, 0)], threads=1, decrypt=False)
    per_output = max(t1, 1e-3)
    n_out = int(max(threads, min(4096, round(target_s / per_output / threads) * threads)))
    outs = [(x // 64, x % 64) for x in range(n_out)]
    _, _, s1 = orc.matmul(A, B, "csr", "per_product", sa, sb, outputs=outs, threads=1, decrypt=False)
    _, _, sT = orc.matmul(A, B, "csr", "per_product", sa, sb, outputs=outs, threads=threads, decrypt=False)
    products = sum(int(np.count_nonzero(A[i])) for (i, _) in outs)
    return {"outputs": n_out, "products": products, "seconds_1_thread": s1, "seconds_T_threads": sT,
            "threads": threads, "speedup": s1 / sT,
            "workload": "N=2^13 64x64x64, A 50% zeros CSR, per-product (Algorithm 1 order)"}


def sweep_leg(torch, sfhe, W, sparsities=(0.0, 0.25, 0.5, 0.75, 0.9)):
    """The sparsity/encoding sweep on the GPU (N = 2^13, 60/40/40-bit data
    primes and one special prime, 64 x 64 x 64, B dense): ms per product for
    the four encodings x both schedules at each sparsity of A, and the
    sparse-over-dense speed-up (the analogue of the paper's runtime against
    sparsity, Sec. 4.2).  One untimed call, then the median of 3."""
    P = W.PARAMS["sweep_n8192"]
    ctx = sfhe.Context(**P)
    ctx.keygen(W.key_seed(2))
    sa, sb = W.enc_seed(2, 0), W.enc_seed(2, 1)
    out = {}
    for sp in sparsities:
        A, B = W.operands(64, 64, 64, sp, W.workload_seed(2))
        EB = ctx.encrypt(B, "dense", sb, 1)
        row = {}
        for enc in ("dense", "naive", "csr", "ell"):
            EA = ctx.encrypt(A, enc, sa, 0)
            for sched in ("lazy", "per_product"):
                tt, st, _, _ = timed(ctx, torch, EA, EB, sched, 3, 1)
                row["%s_%s" % (enc, sched)] = {"ms_median": float(np.median(tt)), "ms_min": float(np.min(tt)),
                                               "products": int(st.products)}
            EA.close()
        for sched in ("lazy", "per_product"):
            row["csr_over_dense_" + sched] = row["dense_" + sched]["ms_median"] / row["csr_" + sched]["ms_median"]
        out["s%02d" % int(round(sp * 100))] = row
        EB.close()
        log("sweep s=%.2f: lazy dense %.2f / csr %.2f ms, per-product dense %.1f / csr %.1f ms" %
            (sp, row["dense_lazy"]["ms_median"], row["csr_lazy"]["ms_median"], row["dense_per_product"]["ms_median"],
             row["csr_per_product"]["ms_median"]))
    ctx.close()
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--sparsity", type=float, default=0.5)
    ap.add_argument("--size", type=int, default=128)
    ap.add_argument("--only", default="", help="comma list of extra legs to run (default all): "
                    "s90,dense,ell,naive,per_product,both,sweep,slots,serve,ctpt,ctpt_launch,cpu,peaks,kstune")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--ctpt-count", type=int, default=32,
                    help="products in the uneven plaintext-weight batch (32 is the workload; fewer for profiling)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="first run one plain device copy of this many MiB (a known-size kernel for "
                         "scaling rocprofv3 FETCH_SIZE / WRITE_SIZE readings)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(the product would shard by output rows, each GPU running this path on its rows)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2503_09184_amd import sfhe
    from paper_2503_09184_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    cfg_id = 3
    P = W.PARAMS["realistic_n16384"]
    n = args.size
    want = set(x for x in args.only.split(",") if x) if args.only else None

    def run(name):
        return (not args.no_extras) and (want is None or name in want)

    if args.calib_copy_mib:
        n_words = args.calib_copy_mib * (1 << 20) // 8
        src = torch.ones(n_words, dtype=torch.int64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: %d MiB read, %d MiB written" % (args.calib_copy_mib, args.calib_copy_mib))
        del src, dst
    peaks = None
    if run("peaks"):
        peaks = measured_peaks(torch, sfhe)
        log("measured peaks %s" % json.dumps(peaks))
    log("setup: context N=2^14, keys")
    ctx = sfhe.Context(**P)
    ctx.keygen(W.key_seed(cfg_id))
    A, Bm = W.operands(n, n, n, args.sparsity, W.workload_seed(cfg_id))
    sa, sb = W.enc_seed(cfg_id, 0), W.enc_seed(cfg_id, 1)
    log("encrypt B (%dx%d dense) and A (CSR, %.0f%% zeros)" % (n, n, 100 * args.sparsity))
    EB = ctx.encrypt(Bm, "dense", sb, 1)
    EA = ctx.encrypt(A, "csr", sa, 0)
    torch.cuda.synchronize()

    log("headline: %d warmup + %d timed steps" % (args.warmup, args.steps))
    ctx.set_profiling(False)
    times, st, C, fp_steps = timed(ctx, torch, EA, EB, "lazy", args.steps, args.warmup, keep_last=True)
    ms = float(np.mean(times))
    products = st.products
    value = products / (ms / 1e3)
    log("headline %.2f ms/step (median %.2f, min %.2f), %d products, %.4g ct-mults/s" %
        (ms, float(np.median(times)), float(np.min(times)), products, value))
    # decrypted error of the headline result (outside the timed region)
    dec = ctx.decrypt(C)
    err = float(np.max(np.abs(dec - A @ Bm)))
    C.close()
    N = ctx.n
    n_fp = int(st.tensor_fp_primes)
    n_int60 = ctx.L - n_fp

    def fp_roofline(fp_list, prods, kernel_name):
        """the fp64 tensor kernel's live timing (hipEvents on the library's
        stream around each launch) against the VALU peaks"""
        fp_ms = sum(m for m, _ in fp_list)
        launches = max(1, sum(k for _, k in fp_list))
        ops = float(prods) * N * n_fp * FP_OPS_PER_PRODUCT * len(fp_list)
        achieved = ops / (fp_ms / 1e3) / 1e12
        peak = VALU_PEAK / 1e12
        r = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "T VALU-op/s", "frac": achieved / peak,
             "kernel": kernel_name, "launches_timed": launches, "ms_per_launch": fp_ms / launches,
             "ops_per_launch": ops / launches, "primes": n_fp}
        if peaks:
            r["peak_measured"] = peaks["fp64_fma_Tops"]
            r["frac_measured"] = achieved / peaks["fp64_fma_Tops"]
        return r

    kname = "tensor_cols_kernel (fp64 residues, primes below 2^42)"
    roofline = fp_roofline(fp_steps, products, kname)
    roofline["traffic"] = measured_traffic()
    # per-step breakdown (one extra, untimed step with every launch group bracketed)
    ctx.set_profiling(True)
    ptimes, pst, _, _ = timed(ctx, torch, EA, EB, "lazy", 1, 0)
    ctx.set_profiling(False)
    breakdown = {"tensor_ms": pst.tensor_ms, "tensor_fp_ms": pst.tensor_fp_ms, "keyswitch_ms": pst.keyswitch_ms,
                 "rescale_ms": pst.rescale_ms, "total_ms": ptimes[0]}
    log("breakdown %s" % json.dumps(breakdown))

    def ks_roofline(ks_ms, keyswitches):
        ops = float(keyswitches) * KS_OPS_PER_OUTPUT
        achieved = ops / (ks_ms / 1e3) / 1e12
        r = {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK / 1e12, "unit": "T VALU-op/s",
             "frac": achieved / (VALU_PEAK / 1e12), "ms": ks_ms, "keyswitches": int(keyswitches),
             "butterflies": float(keyswitches) * KS_BUTTERFLIES_PER_TRANSFORM * (KS_INT_TRANSFORMS + KS_FP_TRANSFORMS),
             "kernels": "ks14_k1/bconv/k2/k3a/k3b (fused key switch and rescale, the lift taken by k3b; N = 2^14)"}
        if peaks:
            # the integer butterflies are bound by the 32-bit/64-bit integer
            # products, the fp64 ones by fp64 issue: the measured peak is the
            # op-weighted mix of the two probes
            w_int = KS_INT_TRANSFORMS * KS_INT_OPS_PER_BUTTERFLY
            w_fp = KS_FP_TRANSFORMS * KS_FP_OPS_PER_BUTTERFLY
            mix = (w_int + w_fp) / (w_int / peaks["mad_u64_u32_Tops"] + w_fp / peaks["fp64_fma_Tops"])
            r["peak_measured"] = mix
            r["frac_measured"] = achieved / mix
        return r

    rooflines = {"keyswitch_rescale_50": ks_roofline(pst.keyswitch_ms, pst.keyswitches)}

    legs = {}

    def leg(name, Amat, enc, sched, steps, warm=1, fp_name=None):
        EAx = ctx.encrypt(Amat, enc, sa, 0)
        tt, stx, _, fpx = timed(ctx, torch, EAx, EB, sched, steps, warm)
        m = float(np.mean(tt))
        legs[name] = {"ms": m, "ms_median": float(np.median(tt)), "ms_min": float(np.min(tt)), "steps": len(tt),
                      "products": int(stx.products), "ct_mults_per_s": stx.products / (m / 1e3),
                      "keyswitches": int(stx.keyswitches)}
        ops = step_ops(stx.products, stx.keyswitches, N, n_fp, n_int60)
        legs[name]["step_valu_ops"] = ops
        legs[name]["step_frac_of_valu_peak"] = ops / (float(np.median(tt)) / 1e3) / VALU_PEAK
        if fp_name:
            rooflines[fp_name] = fp_roofline(fpx, stx.products, kname)
        EAx.close()
        log("%s: %.2f ms (median %.2f, min %.2f), %d products" % (name, m, legs[name]["ms_median"],
                                                                 legs[name]["ms_min"], stx.products))
        return stx

    # the key-switch slice the tuner chose (at the first product) against
    # the untuned default of 2048 outputs per launch group
    ks_slice, ks_streams, ks_us, ks_us2 = ctx.ks_tuning()
    ks_tuning = {"slice_in_use": ks_slice, "streams_in_use": ks_streams,
                 "us_per_output_one_stream": {str(k): v for k, v in ks_us.items()},
                 "us_per_output_two_streams": {str(k): v for k, v in ks_us2.items()}}
    if run("kstune") and (ks_slice, ks_streams) != (2048, 1) and ks_slice != 0:
        ctx.set_ks_slice(2048, 1)
        tt, _, _, _ = timed(ctx, torch, EA, EB, "lazy", max(2, min(args.steps, 5)), 1)
        ctx.set_ks_slice(-1)
        ks_tuning["untuned_2048_one_stream_ms_median"] = float(np.median(tt))
        ks_tuning["tuned_ms_median"] = float(np.median(times))
        log("key switch: tuned %d x %d stream(s) (%.2f ms/step) vs 2048 x 1 (%.2f ms/step)" %
            (ks_slice, ks_streams, float(np.median(times)), float(np.median(tt))))
    legs["lazy_csr_50"] = {"ms": ms, "ms_median": float(np.median(times)), "ms_min": float(np.min(times)),
                           "steps": len(times), "products": int(products), "ct_mults_per_s": value,
                           "keyswitches": int(st.keyswitches)}
    ops50 = step_ops(products, st.keyswitches, N, n_fp, n_int60)
    legs["lazy_csr_50"]["step_valu_ops"] = ops50
    legs["lazy_csr_50"]["step_frac_of_valu_peak"] = ops50 / (float(np.median(times)) / 1e3) / VALU_PEAK
    if run("ell"):
        leg("lazy_ell_50", A, "ell", "lazy", args.steps)
    if run("naive"):
        leg("lazy_naive_50", A, "naive", "lazy", args.steps)
    if run("dense"):
        leg("lazy_dense_same_operands", A, "dense", "lazy", args.steps, fp_name="tensor_fp_dense")
    A90 = None
    if run("s90"):
        A90, _ = W.operands(n, n, n, 0.9, W.workload_seed(cfg_id))
        leg("lazy_csr_90", A90, "csr", "lazy", args.steps, fp_name="tensor_fp_90")
        if run("dense"):
            leg("lazy_dense_90_operands", A90, "dense", "lazy", max(1, min(3, args.steps)))
    if run("per_product"):
        # Algorithm 1's order: one warm-up, then the median and min of 3
        leg("per_product_csr_50", A, "csr", "per_product", 3)
        if A90 is not None:
            leg("per_product_csr_90", A90, "csr", "per_product", 3)
    if run("both"):
        # both operands sparse (the paper's own setting): B with half its
        # entries zero, as a ReLU leaves activations, CSR on both sides
        Bz = Bm.copy()
        Bz[np.random.default_rng(W.workload_seed(cfg_id) + 5).random(Bz.shape) < 0.5] = 0.0
        EBz = ctx.encrypt(Bz, "csr", sb, 1)
        EAx = ctx.encrypt(A, "csr", sa, 0)
        tt, stx, _, _ = timed(ctx, torch, EAx, EBz, "lazy", args.steps, 1)
        m = float(np.mean(tt))
        legs["lazy_csr_both_50"] = {"ms": m, "ms_median": float(np.median(tt)), "products": int(stx.products),
                                    "ct_mults_per_s": stx.products / (m / 1e3), "keyswitches": int(stx.keyswitches),
                                    "b_zero_fraction": float(np.mean(Bz == 0.0))}
        log("lazy_csr_both_50: %.2f ms, %d products" % (m, stx.products))
        EAx.close()
        EBz.close()
    # per-kernel breakdown of the 90% step
    if A90 is not None:
        EA9 = ctx.encrypt(A90, "csr", sa, 0)
        ctx.set_profiling(True)
        t9, st9, _, _ = timed(ctx, torch, EA9, EB, "lazy", 1, 0)
        ctx.set_profiling(False)
        breakdown["s90"] = {"tensor_ms": st9.tensor_ms, "tensor_fp_ms": st9.tensor_fp_ms,
                            "keyswitch_ms": st9.keyswitch_ms, "rescale_ms": st9.rescale_ms, "total_ms": t9[0]}
        rooflines["keyswitch_rescale_90"] = ks_roofline(st9.keyswitch_ms, st9.keyswitches)
        EA9.close()
    EA.close()
    EB.close()
    torch.cuda.empty_cache()
    if run("sweep"):
        log("sparsity/encoding sweep at N = 2^13 (64 x 64 x 64)")
        legs["sweep_n8192"] = sweep_leg(torch, sfhe, W)
    if run("slots"):
        log("chunks of 8 values per ciphertext: Algorithm 1 with rotations and the slot-0 mask")
        legs["slots8_lazy_csr_50"] = slots_leg(ctx, torch, A, Bm, sa, sb, 8)
        log("slots8: %.1f ms, %d products, %d key switches and rotations, err %.2e" %
            (legs["slots8_lazy_csr_50"]["ms"], legs["slots8_lazy_csr_50"]["products"],
             legs["slots8_lazy_csr_50"]["keyswitches_and_rotations"], legs["slots8_lazy_csr_50"]["max_abs_err_vs_fp64"]))
        # both schedules on a 32-row slice of the same operands (Algorithm 1's
        # own order rotates every product to its output slot: 8x the rotations)
        for sched in ("lazy", "per_product"):
            name = "slots8_%s_csr_50_32x128x128" % sched
            legs[name] = slots_leg(ctx, torch, A[:32], Bm, sa, sb, 8, sched)
            log("%s: %.1f ms, %d products" % (name, legs[name]["ms"], legs[name]["products"]))
    if run("serve"):
        log("serving: Poisson arrivals of encrypted MLP-layer requests")
        legs["serving"] = serving_leg(torch, sfhe, W)
        log("serving (%s): p50 %.1f ms, p99 %.1f ms, %.4g ct-pt mults/s, %d batches" %
            (legs["serving"]["policy"], legs["serving"]["latency_ms_p50"], legs["serving"]["latency_ms_p99"],
             legs["serving"]["ctpt_mults_per_s"], legs["serving"]["batches"]))
    if run("ctpt"):
        log("plaintext weights x encrypted values: uneven batch of 32 products")
        legs["ctpt_uneven_batch"] = ctpt_leg(torch, sfhe, W, args.ctpt_count)
        log("ctpt: %d products in %.1f ms, %.4g ct-pt mults/s" %
            (legs["ctpt_uneven_batch"]["products"], legs["ctpt_uneven_batch"]["ms"],
             legs["ctpt_uneven_batch"]["ctpt_mults_per_s"]))
    if run("ctpt_launch"):
        legs["ctpt_launch_forms"] = ctpt_launch_leg(torch, sfhe, W, args.ctpt_count)

    cpu = None
    if not args.no_cpu and run("cpu"):
        affinity = len(os.sched_getaffinity(0))
        # at most 16 threads: the host cores that go with one GPU, whatever the affinity mask shows
        threads = max(1, min(affinity, 16))
        log("cpu baseline: oracle on %d threads (%d in the affinity mask)" % (threads, affinity))
        cpu = cpu_baseline(P, A, Bm, cfg_id, threads)
        cpu["affinity_cores"] = affinity
        log("cpu baseline %.4g ct-mults/s" % cpu["value"])
        cpu["thread_scaling"] = cpu_thread_scaling(threads)
        log("oracle thread speed-up %.2fx on %d threads" % (cpu["thread_scaling"]["speedup"], threads))

    speedups = {}
    if "lazy_dense_same_operands" in legs:
        speedups["sparse50_over_dense"] = legs["lazy_dense_same_operands"]["ms"] / ms
    if "lazy_csr_90" in legs and "lazy_dense_90_operands" in legs:
        speedups["sparse90_over_dense"] = legs["lazy_dense_90_operands"]["ms"] / legs["lazy_csr_90"]["ms"]
    if "per_product_csr_50" in legs:
        speedups["lazy_over_per_product_50"] = legs["per_product_csr_50"]["ms_median"] / float(np.median(times))
    if "per_product_csr_90" in legs and "lazy_csr_90" in legs:
        speedups["lazy_over_per_product_90"] = legs["per_product_csr_90"]["ms_median"] / legs["lazy_csr_90"]["ms_median"]
    if "slots8_per_product_csr_50_32x128x128" in legs:
        speedups["slots8_lazy_over_per_product_32x128x128"] = (legs["slots8_per_product_csr_50_32x128x128"]["ms"] /
                                                               legs["slots8_lazy_csr_50_32x128x128"]["ms"])
    if "lazy_csr_both_50" in legs and "lazy_dense_same_operands" in legs:
        # the dense schedule's time does not depend on the values
        speedups["both_sparse50_over_dense"] = legs["lazy_dense_same_operands"]["ms"] / legs["lazy_csr_both_50"]["ms"]

    out = {
        "metric": "ms per encrypted 128x128x128 matmul @50%/90% sparsity; ct-mults/s vs dense",
        "value": value,
        "unit": "ct-mults/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "ms_per_step_median": float(np.median(times)),
        "ms_per_step_min": float(np.min(times)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64/f64",
        "data": "synthetic",
        "config": {"workload": "encrypted %dx%dx%d matmul, A %.0f%% unstructured sparsity (CSR), B dense, "
                               "RNS-CKKS N=2^14, 5 data + 3 special primes, dnum=2, lazy relinearisation"
                               % (n, n, n, 100 * args.sparsity),
                   "products_per_step": int(products), "parallelism": "single GPU"},
        "max_abs_err_vs_fp64": err,
        "breakdown_ms": breakdown,
        "legs": legs,
        "speedups": speedups,
        "roofline": roofline,
        "rooflines": rooflines,
        "measured_peaks": peaks,
        "ntt_designs": {d: {"used": ctx.ntt_tuning(d == "inverse")[0], "us_per_row": ctx.ntt_tuning(d == "inverse")[1]}
                        for d in ("forward", "inverse")},
        "ks_slice_tuning": ks_tuning,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
