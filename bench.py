"""Benchmark: packed ct x ct h=64 matrix products per second at N = 2^15 on one MI355X.

Workload (one "step"): a batch of B independent h=64 products HE-MatMult (Alg. 3 with
the App. B baby-step/giant-step split) on the N=2^15 ring with Q = 60 + 13 x 45 bits,
P = 3 x 60 + 56 bits, dnum 3, scale 2^45; inputs are fresh encryptions at the top
level (13) of matrices with entries uniform in [-1, 1], resident in HBM before the
timed region.  The plain path (one he_matmul at a time) is timed beside it.

Prints one JSON line: the headline rate and its roofline, the step's traffic, the per-kernel
breakdown, the other configurations and the oracle baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "ct×ct h=64 HE-matmuls/s at N=2^15 vs plain path; p50/p99 serve latency"
HBM_PEAK_GBS = 8000.0
# ALU peak of the NTT butterfly on gfx950, from unit counts and clock: 256 CUs x 4 SIMD
# x 16 lanes x 2.4 GHz = 39.32 T VALU lane-instructions/s.  One lazy Shoup butterfly
# (x' = x - 2q if x >= 2q; t = x1 w - floor(x1 w' / 2^64) q; (x' + t, x' - t + 2q)) is 28 VALU
# instructions on gfx950: 10 integer multiplies (v_mad_u64_u32, v_mul_lo_u32, v_mul_hi_u32)
# and 18 adds/subtracts/compares/selects/moves, all issued at the full rate.
# The limbs of primes below 2^46 run FP64 butterflies instead: hi = x w, lo = fma(x, w, -hi),
# c = rint(x fl(w/q)), t = fma(-c, q, hi) + lo, then x + t and x - t: 8 VALU instructions
# (v_mul/v_fma/v_rndne/v_add_f64, full rate on gfx950).  A transform launch is bound by
# whichever floor is larger: its algorithmic bytes at 8 TB/s, or its butterflies' VALU
# instructions at the VALU rate.
VALU_LANE_OPS = 256 * 4 * 16 * 2.4e9
BFLY_INSTR = 28
FP64_BFLY_INSTR = 8
NTT_KERNELS = ("ntt_fwd_cols", "ntt_fwd_rows", "ntt_inv_rows", "ntt_inv_cols")


def measured_traffic(kernel):
    """HBM bytes per launch from the committed PMC summary, if the kernel sources are the
    ones the counters were taken on (else None)."""
    import hashlib
    f = os.path.join(ROOT, "profiles", f"{kernel}_c3_h64_batch16.traffic.json")
    if not os.path.exists(f):
        return None
    rec = json.load(open(f))
    h = hashlib.sha256()
    for src in rec["sources"]:
        h.update(open(os.path.join(ROOT, src), "rb").read())
    return rec["traffic_bytes_per_launch"] if h.hexdigest() == rec["sources_sha256"] else None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


SCHEDULES = {"each": 0, "once": 1, "once+hoist": 3, "once+hoist+late": 7, "fast": 15}
SCHEDULE_TEXT = {0: "relinearise every Step-3 product (Alg. 3 as printed)",
                 1: "relinearise once per product",
                 3: "relinearise once; one ModDown per Step-2 mask pair",
                 7: "relinearise once; one ModDown per Step-2 mask pair; A^(k) rescaled late (two final rescales)",
                 15: "relinearise once per Step-3 block; one ModDown per Step-2 mask pair; A^(k) rescaled late; "
                     "Step 3 split into 16 baby x 4 giant steps"}


def host_cpu():
    """the host's CPU model and core counts (lscpu), and the threads this process may use"""
    import subprocess
    info = {"model": None, "sockets": None, "cores_per_socket": None, "threads_per_core": None}
    try:
        out = subprocess.check_output(["lscpu"], text=True, env=dict(os.environ, LC_ALL="C"))
        for line in out.splitlines():
            k, _, v = line.partition(":")
            v = v.strip()
            if k == "Model name":
                info["model"] = v
            elif k == "Socket(s)":
                info["sockets"] = int(v)
            elif k == "Core(s) per socket":
                info["cores_per_socket"] = int(v)
            elif k == "Thread(s) per core":
                info["threads_per_core"] = int(v)
    except (OSError, ValueError, subprocess.CalledProcessError):
        pass
    phys = info["sockets"] * info["cores_per_socket"] if info["sockets"] and info["cores_per_socket"] else None
    return {"cpu_model": info["model"], "physical_cores": phys, "nproc": os.cpu_count(),
            "usable_threads": len(os.sched_getaffinity(0))}


def _median3(fn):
    ts = []
    for _ in range(3):
        t0 = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t0)
    return sorted(ts)[1]


def cpu_baseline(prm, flags):
    """The oracle (plain scalar C, OpenMP over limbs) on the host, as it stands.  Bounded sample:
    the benchmark's own unit, one C3 h=64 product from level 13 under the same schedule, timed
    directly three times at every usable thread (median; the rotation keys and masks come from
    an untimed first product).  Beside it, one directly timed C3 product for h = 16 and 32 and
    one C2 h=64 product, and a one-thread figure from an operation-level model: each operation
    the product performs, timed on the N=2^15 ring at level 12 (median of three, at one thread
    and at every thread), weighted by the product's operation counts under the same schedule
    (counted exactly by running the oracle's product on a 2^13 ring, where the counts are the
    same); the all-thread model against the direct timing checks the model."""
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import oracle as O
    from paper_2207_04620_amd import inputs as I

    host = host_cpu()
    nthr = host["usable_threads"]

    def direct(p, h, reps):
        o = O.Ctx.from_params(p, threads=nthr)
        A, B = I.matrix_pair(3, h)
        a, b = o.encrypt(A.ravel(), nonce=1), o.encrypt(B.ravel(), nonce=2)
        o.matmul(a, b, h, flags)  # rotation keys and masks for h (not timed)
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            o.matmul(a, b, h, flags)
            ts.append(time.perf_counter() - t0)
        return sorted(ts)[len(ts) // 2]

    log("cpu baseline: C3 h=64 products on the oracle")
    t64 = direct(prm, 64, 3)
    per_h = {"16": round(direct(prm, 16, 1), 3), "32": round(direct(prm, 32, 1), 3), "64": round(t64, 3)}
    log("cpu baseline: C2 h=64 product")
    c2_64 = direct(I.C2, 64, 1)

    c = O.Ctx(13, [50, 40, 40, 40, 40], [50, 50], 2, 40.0, 7, threads=nthr)
    A, B = I.matrix_pair(3, 64)
    a, b = c.encrypt(A.ravel(), nonce=1), c.encrypt(B.ravel(), nonce=2)
    c.reset_counters()
    c.matmul(a, b, 64, flags)
    cnt = c.counters()

    def op_times(threads):
        o = O.Ctx.from_params(prm, threads=threads)
        A, B = I.matrix_pair(5, 64)
        lvl = prm.max_level - 1
        a, b = o.encrypt(A.ravel(), level=lvl, nonce=1), o.encrypt(B.ravel(), level=lvl, nonce=2)
        pt = o.encode(np.ones(8))[0]
        o.rotate(a, 1)  # the key (not timed)
        t = o.tensor(a, b)
        o.relin(t)      # the relinearisation key is made with the context
        return {"rot": _median3(lambda: o.rotate(a, 1)),
                "relin": _median3(lambda: o.relin(t)),
                "mul_pt": _median3(lambda: o.mul_plain(a, pt, o.scale)),
                "mul_ct": _median3(lambda: o.tensor(a, b)),
                "add": _median3(lambda: o.add(a, b)),
                "rescale": _median3(lambda: o.rescale(a))}

    def model(t):
        relins = cnt["keyswitch"] - cnt["rot"] if cnt["keyswitch"] >= cnt["rot"] else cnt["mul_ct"]
        return (cnt["rot"] * t["rot"] + max(0, relins) * t["relin"] + cnt["mul_pt"] * t["mul_pt"] +
                cnt["mul_ct"] * t["mul_ct"] + cnt["add"] * t["add"] + cnt["rescale"] * t["rescale"])

    log("cpu baseline: operation-level model at one thread")
    t_all, t_one = op_times(nthr), op_times(1)
    est_all, est_one = model(t_all), model(t_one)
    return {"value": round(1.0 / t64, 5), "unit": "HE-matmuls/s", "cores": nthr, "kind": "oracle",
            "sample": f"one C3 h=64 product from level 13 under the same schedule, timed directly three times at "
                      f"{nthr} threads (median); keys and masks from an untimed first product",
            "h64_seconds": round(t64, 3), "c3_seconds_by_h": per_h, "c2_h64_seconds": round(c2_64, 3),
            "value_1_thread": round(1.0 / est_one, 6), **host,
            "model": {"note": "each operation of the h=64 product timed on the N=2^15 ring at level 12 (median of "
                              f"3), weighted by the product's operation counts ({cnt['rot']} rotations, "
                              f"{cnt['keyswitch']} key switches, {cnt['mul_pt']} Mul_pt, {cnt['mul_ct']} Mul_ct, "
                              f"{cnt['rescale']} rescales)",
                      "h64_seconds_all_threads": round(est_all, 2), "h64_seconds_1_thread": round(est_one, 2),
                      "op_seconds_all_threads": {k: round(v, 4) for k, v in t_all.items()},
                      "op_seconds_1_thread": {k: round(v, 4) for k, v in t_one.items()}}}


def mixed_leg(he, I, prm, sched, stream, count):
    """The mixed-batch configuration: count products with h uniform over {16, 32, 64} and
    starting levels uniform over [3, 13] (inputs.batch_mix, seed 3) in one batched call.
    Four encrypted pairs per h are shared by the members (level drops of them)."""
    ctx = he.Context(prm, h_list=[16, 32, 64], stream=stream.cuda_stream, schedule=sched)
    mix = I.batch_mix(3, count)
    base = {h: [(ctx.encrypt(A.ravel(), nonce=10 * h + 2 * i), ctx.encrypt(B.ravel(), nonce=10 * h + 2 * i + 1))
                for i, (A, B) in enumerate(I.matrix_pair(700 + h + i, h) for i in range(4))] for h in (16, 32, 64)}
    As, Bs = [], []
    for i, (h, lv) in enumerate(mix):
        a, b = base[h][i % 4]
        As.append(ctx.drop(a, lv))
        Bs.append(ctx.drop(b, lv))
    hs = [h for h, _ in mix]
    ctx.matmul_batch(As, Bs, hs)
    ctx.sync()
    t0 = time.perf_counter()
    ctx.matmul_batch(As, Bs, hs)
    ctx.sync()
    dt = time.perf_counter() - t0
    ctx.close()
    counts = {h: hs.count(h) for h in (16, 32, 64)}
    return {"products": count, "h_counts": counts, "levels": "uniform over [3, 13]",
            "matmuls_per_s": round(count / dt, 3), "ms": round(dt * 1e3, 1)}


def c4_leg(he, I, sched, stream, count):
    """The sign/ReLU configuration on the N=2^16 ring: count ciphertexts of 32 x 32 inputs
    (|x| in [2^-8, 1], random sign), ReLU by g_3^(3) in one batched call, then one h=32
    product of each result with an encrypted W in a second batched call.  Eight distinct
    encrypted inputs are shared by the members."""
    prm = I.C4
    ctx = he.Context(prm, h_list=[32], stream=stream.cuda_stream, schedule=sched)
    X = I.sign_inputs(4, 8, 32)
    xs = [ctx.encrypt(X[i % 8].ravel(), nonce=i + 1) for i in range(8)]
    xs = [xs[i % 8] for i in range(count)]
    W = np.random.default_rng(4).uniform(-1.0, 1.0, (32, 32))
    ys = ctx.sign_approx_batch(xs[:8], 3, 3, he.RELU)  # warm-up
    lvl = ys[0].info()[0]
    w = ctx.encrypt(W.ravel(), level=lvl, nonce=1000)
    ctx.matmul_batch(ys, [w] * 8, [32] * 8)
    ctx.sync()
    t0 = time.perf_counter()
    ys = ctx.sign_approx_batch(xs, 3, 3, he.RELU)
    ctx.sync()
    t1 = time.perf_counter()
    ms = ctx.matmul_batch(ys, [w] * count, [32] * count)
    ctx.sync()
    t2 = time.perf_counter()
    g3 = lambda v: (35 * v - 35 * v ** 3 + 21 * v ** 5 - 5 * v ** 7) / 16  # noqa: E731
    relu = (X[0] + X[0] * g3(g3(g3(X[0])))) / 2
    err = float(np.abs(ctx.decrypt(ms[0], 1024).reshape(32, 32) - relu @ W).max())
    ctx.close()
    return {"ciphertexts": count, "relu_per_s": round(count / (t1 - t0), 2),
            "h32_matmuls_per_s": round(count / (t2 - t1), 2),
            "end_to_end_per_s": round(count / (t2 - t0), 2), "max_abs_error": err}


def serve_rings_leg(he, I, sched, nreq, load):
    """The serving configuration across rings: one server per context (N = 2^14, 2^15,
    2^16), mixed requests (60% products with h uniform over {8, 16, 32, 64, 128}; 25% sign or
    ReLU with d = 3 and k uniform over 1..4 (depth 3..13); 5% of depth 1 and 2 (x^2, x . x^2);
    10% the N=2^16 ReLU k = 3, so that the largest ring serves too) routed to the smallest ring
    that holds them.  The burst capacity is measured with nreq requests at once; the Poisson
    capacity, the highest Poisson arrival rate the servers keep up with, by bisection; latency
    with Poisson arrivals (seed 5) at 0.5, 0.8 and 0.95 x the Poisson capacity, from scheduled
    arrival to completion."""
    rings = [he.Context(I.C2, h_list=[8, 16, 32, 64], schedule=sched),
             he.Context(I.C3, h_list=[128], schedule=sched),
             he.Context(I.C4, h_list=[], schedule=sched)]
    rng = np.random.default_rng(5)
    kinds = []
    for _ in range(nreq):
        u = rng.random()
        if u < 0.60:
            kinds.append(("mm", int(rng.choice([8, 16, 32, 64, 128]))))
        elif u < 0.85:
            kinds.append(("sign", 3, int(rng.integers(1, 5)), int(rng.integers(0, 2))))
        elif u < 0.90:  # depth 1 and 2: a square, a square and a product
            kinds.append(("pow", int(rng.integers(2, 4))))
        else:
            kinds.append(("c4relu", 3, 3, he.RELU))
    inputs = {}

    def operands(w):
        if w[0] == "mm":
            ctx = he.smallest_ring(rings, h=w[1], depth=3)
        elif w[0] == "sign":
            ctx = he.smallest_ring(rings, h=32, depth=he.sign_depth(w[1], w[2], w[3]))
        elif w[0] == "pow":
            ctx = he.smallest_ring(rings, h=32, depth=w[1] - 1)
        else:
            ctx = rings[2]
        key = (id(ctx), w[0] if w[0] == "mm" else "x", w[1] if w[0] == "mm" else 32)
        if key not in inputs:
            h = w[1] if w[0] == "mm" else 32
            if w[0] == "mm":
                A, B = I.matrix_pair(900 + h, h)
                inputs[key] = (ctx.encrypt(A.ravel(), nonce=1), ctx.encrypt(B.ravel(), nonce=2))
            else:
                inputs[key] = (ctx.encrypt(I.sign_inputs(901, 1, 32)[0].ravel(), nonce=3), None)
        return ctx, inputs[key]

    plan = [(w,) + operands(w) for w in kinds]
    servers = {id(c): he.Server(c, max_batch=16, min_batch=8, max_wait_us=40000) for c in rings}

    def submit(w, ctx, ops):
        srv = servers[id(ctx)]
        if w[0] == "mm":
            return srv, srv.submit(he.REQ_MATMUL, ops[0], ops[1], h=w[1])
        if w[0] == "pow":
            return srv, srv.submit(he.REQ_POWER, ops[0], k=w[1])
        return srv, srv.submit(he.REQ_SIGN, ops[0], d=w[1], k=w[2], mode=w[3])

    def drain(tk, late, arrivals):
        """latency = submit delay + the server's submit -> completion time (taken after the
        stream synchronises); completion offsets give the served rate"""
        lat = {}
        while len(lat) < len(tk):
            for j, (srv, t) in enumerate(tk):
                if j not in lat:
                    r = srv.poll(t)
                    if r is not None:
                        lat[j] = late[j] + r[1]
            time.sleep(0.0005)
        return lat, float(max(arrivals[j] + lat[j] for j in lat))

    def submit_all(arrivals):
        tk, late = [], []
        t0 = time.perf_counter()
        for j, p in enumerate(plan):
            while time.perf_counter() - t0 < arrivals[j]:
                time.sleep(0.0002)
            late.append((time.perf_counter() - t0) - arrivals[j])
            tk.append(submit(*p))
        return tk, late

    def run_at(rate):
        arrivals = I.poisson_arrivals(5, rate, nreq)
        tk, late = submit_all(arrivals)
        lat, span = drain(tk, late, arrivals)
        lats = np.array([lat[j] for j in range(nreq)])
        by = {}
        for name, sel in (("matmul", lambda w: w[0] == "mm"), ("sign", lambda w: w[0] == "sign"),
                          ("power", lambda w: w[0] == "pow"), ("c4_relu", lambda w: w[0] == "c4relu")):
            v = np.array([lat[j] for j in range(nreq) if sel(kinds[j])])
            if v.size:
                by[name] = {"n": int(v.size), "p50_ms": round(float(np.percentile(v, 50)) * 1e3, 1),
                            "p99_ms": round(float(np.percentile(v, 99)) * 1e3, 1)}
        return {"arrival_rate_per_s": round(rate, 1), "served_per_s": round(nreq / span, 1),
                "p50_ms": round(float(np.percentile(lats, 50)) * 1e3, 1),
                "p99_ms": round(float(np.percentile(lats, 99)) * 1e3, 1), "by_type": by}

    # burst capacity: every request at t = 0
    tk, late = submit_all([0.0] * nreq)
    _, span = drain(tk, late, [0.0] * nreq)
    capacity = nreq / span
    # Poisson capacity: the highest arrival rate the servers keep up with (served at least at the
    # arrival rate, p99 within 3 x p50), by bisection between 0.6 and 1.0 x the burst capacity
    lo, hi, search = 0.6, 1.0, []
    for _ in range(3):
        mid = 0.5 * (lo + hi)
        r = run_at(mid * capacity)
        ok = r["served_per_s"] >= r["arrival_rate_per_s"] and r["p99_ms"] <= 3 * r["p50_ms"]
        search.append({"fraction_of_burst": round(mid, 3), "served_per_s": r["served_per_s"],
                       "p50_ms": r["p50_ms"], "p99_ms": r["p99_ms"], "kept_up": ok})
        lo, hi = (mid, hi) if ok else (lo, mid)
    pcap = lo * capacity
    runs = []
    for ld in sorted({0.5, 0.95, load}):
        runs.append({"load": ld, **run_at(ld * pcap)})
    for srv in servers.values():
        srv.stop()
    for c in rings:
        c.close()
    return {"requests": nreq, "rings": "N=2^14 (C2), 2^15 (C3), 2^16 (C4)", "types": len(set(kinds)),
            "batching_window": {"min_batch": 8, "max_wait_ms": 40, "per_type": True},
            "burst_capacity_per_s": round(capacity, 1), "poisson_capacity_per_s": round(pcap, 1),
            "poisson_capacity_search": search,
            "loads": "fractions of the Poisson capacity", "poisson": runs}


def shapes_leg(he, I, prm, sched, stream, batch):
    """The other matrix operations of the paper on the same ring, each a batch of 'batch'
    independent ciphertexts: four h=64 products packed per ciphertext pair (iota_4, App. E),
    a 16 x 64 by 64 x 64 product (HE-RMatMult, Alg. 6), and h=64 transposition (App. C)."""
    ctx = he.Context(prm, h_list=[], stream=stream.cuda_stream, schedule=sched)
    out = {}
    rng = np.random.default_rng(6)
    packed = [(he.pack_beta([rng.uniform(-1, 1, (64, 64)) for _ in range(4)]),
               he.pack_beta([rng.uniform(-1, 1, (64, 64)) for _ in range(4)])) for _ in range(4)]
    As = [ctx.encrypt(packed[i % 4][0], nonce=2 * i) for i in range(batch)]
    Bs = [ctx.encrypt(packed[i % 4][1], nonce=2 * i + 1) for i in range(batch)]
    for name, shape, count in (("packed_beta4_h64", (64, 64, 4), 4), ("rect_t16_h64", (64, 16, 1), 1)):
        ctx.matmul_batch_ex(As, Bs, [shape] * batch)
        ctx.sync()
        t0 = time.perf_counter()
        ctx.matmul_batch_ex(As, Bs, [shape] * batch)
        ctx.sync()
        dt = time.perf_counter() - t0
        out[name] = {"ciphertext_products_per_s": round(batch / dt, 2),
                     "matrix_products_per_s": round(batch * count / dt, 2), "ms_per_batch": round(dt * 1e3, 1)}
    ctx.transpose_batch(As, 64, 1)
    ctx.sync()
    t0 = time.perf_counter()
    ctx.transpose_batch(As, 64, 1)
    ctx.sync()
    dt = time.perf_counter() - t0
    out["transpose_h64"] = {"transposes_per_s": round(batch / dt, 2), "ms_per_batch": round(dt * 1e3, 1)}
    ctx.close()
    out["batch"] = batch
    return out


def hbm_probe(torch, ctx, words=1 << 27, reps=20):
    """What a plain streaming kernel moves through HBM on this device (he_stream_probe: one pass
    of 16-byte nontemporal accesses, 1 GiB per stream): read only, copy (one read and one write
    stream) and two read streams with one write stream (the ModDown row pass's mix), in GB/s of
    bytes moved"""
    a = torch.empty(words, dtype=torch.int64, device="cuda")
    b = torch.empty(words, dtype=torch.int64, device="cuda")
    c = torch.empty(words, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    out = {}
    for name, pattern, streams in (("read", 0, 1), ("copy", 1, 2), ("two_reads_one_write", 2, 3)):
        ms = ctx.stream_probe(pattern, a, b if pattern == 2 else None, c, reps)
        out[f"{name}_GB/s"] = round(streams * 8 * words / (ms * 1e-3) / 1e9, 1)
    out["bytes_per_stream"] = 8 * words
    out["note"] = ("he_stream_probe: one pass of 16-byte nontemporal accesses, mean of 20 launches after one; "
                   "the row pass reads two streams and writes one")
    del a, b, c
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--schedule", choices=list(SCHEDULES), default="fast",
                    help="schedule flags of the product (each: relinearise every Step-3 product; once: "
                         "relinearise the sum; +hoist: one ModDown per Step-2 mask pair; fast: also rescale "
                         "A^(k) late)")
    ap.add_argument("--plain-iters", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="keep the default scheduling knobs")
    ap.add_argument("--no-graph", action="store_true", help="skip the HIP-graph replay of the batched step")
    ap.add_argument("--no-other", action="store_true", help="skip timing the other schedules")
    ap.add_argument("--mix", type=int, default=256, help="mixed-batch products (0: skip)")
    ap.add_argument("--c4", type=int, default=128, help="ciphertexts of the N=2^16 ReLU + h=32 leg (0: skip)")
    ap.add_argument("--serve-rings", type=int, default=2000, help="requests of the cross-ring serving leg (0: skip)")
    ap.add_argument("--no-shapes", action="store_true", help="skip the packed / rectangular / transpose leg")
    ap.add_argument("--no-probe", action="store_true", help="skip the streaming-bandwidth probe")
    ap.add_argument("--roofline-steps", type=int, default=1,
                    help="last timed steps whose dominant-kernel launches carry timing events")
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--serve-load", type=float, default=0.8, help="arrival rate / batched capacity")
    ap.add_argument("--serve-min-batch", type=int, default=8)
    ap.add_argument("--serve-max-wait-ms", type=float, default=60.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the packed product is sharded by "
              "request across GPUs with no exchange step, so N GPUs give N independent copies of this number.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2207_04620_amd import he, inputs as I

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    prm = I.C3
    h = 64
    log("context C3 (keys + masks for h=64)")
    t0 = time.perf_counter()
    sched = SCHEDULES[args.schedule]
    ctx = he.Context(prm, h_list=[h], stream=stream.cuda_stream, schedule=sched)
    log(f"context ready in {time.perf_counter() - t0:.1f} s")
    level = prm.max_level
    As, Bs = [], []
    for i in range(args.batch):
        A, B = I.matrix_pair(1000 + i, h)
        As.append(ctx.encrypt(A.ravel(), level=level, nonce=2 * i))
        Bs.append(ctx.encrypt(B.ravel(), level=level, nonce=2 * i + 1))
    ctx.sync()

    # plain path: one product at a time
    plain_s = float("nan")
    if args.plain_iters > 0:
        log("plain path")
        ctx.matmul(As[0], Bs[0], h)
        ctx.sync()
        t0 = time.perf_counter()
        for i in range(args.plain_iters):
            ctx.matmul(As[i % args.batch], Bs[i % args.batch], h)
        ctx.sync()
        plain_s = (time.perf_counter() - t0) / args.plain_iters
        log(f"plain {plain_s * 1e3:.1f} ms per product")

    # the autotuner's choice of the scheduling knobs for this shape (untimed; results do not
    # depend on it)
    tune = None
    if not args.no_tune:
        log("autotune")
        tune = ctx.autotune(h, level, args.batch)
        log(f"autotune: {tune['chosen']} ({tune['source']})")
        ch = tune["chosen"]
        if ch["max_group"] < args.batch:
            # a split batch runs its groups concurrently on two streams, where one launch's
            # duration no longer measures that kernel; the timed step stays one lockstep group
            # (the tuned sets per launch and overlap), the split's own time is in the report
            split = min(c["ms"] for c in tune["candidates"] if c["max_group"] < args.batch)
            one = min((c for c in tune["candidates"] if c["max_group"] == args.batch), key=lambda c: c["ms"])
            tune["split_batch_products_per_s"] = round(args.batch / (split * 1e-3), 2)
            ctx.set_tuning(one["pair_batch"], args.batch, one["overlap"], ch["concurrent_groups"])
            tune["timed_with"] = ctx.tuning()

    # batched path
    log("batched path: warmup")
    for _ in range(args.warmup):
        ctx.matmul_batch(As, Bs, [h] * args.batch)
    ctx.sync()
    # one untimed pass with every launch bracketed by events: per-kernel breakdown and the
    # dominant kernel (events on ~2.6k launches per step slow the step by ~10 %)
    ctx.profile(True)
    t0 = time.perf_counter()
    ctx.matmul_batch(As, Bs, [h] * args.batch)
    ctx.sync()
    prof_elapsed = time.perf_counter() - t0
    ctx.profile(False)
    prof_all = ctx.profile_report()
    dom = max(prof_all, key=lambda k: prof_all[k]["ms"])
    log(f"profiled pass {prof_elapsed * 1e3:.1f} ms; dominant kernel {dom}")
    # timed region: events only around the dominant kernel's launches, and only in the last
    # roofline_steps steps (each event pair cost ~4 us of the step: bracketing every launch of
    # every timed step slowed the measured step by ~1.5 %)
    torch.cuda.synchronize()
    ev_from = args.steps - max(1, min(args.steps, args.roofline_steps))
    t0 = time.perf_counter()
    out = None
    for s in range(args.steps):
        if s == ev_from:
            ctx.profile(True, only=dom)
        out = ctx.matmul_batch(As, Bs, [h] * args.batch)
        log(f"step {s + 1}/{args.steps} issued")
    ctx.sync()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ctx.profile(False)
    prof = ctx.profile_report()
    step_ms = elapsed / args.steps * 1e3
    value = args.batch * args.steps / elapsed
    err = float(np.abs(ctx.decrypt(out[0], h * h).reshape(h, h) - np.dot(*I.matrix_pair(1000, h))).max())
    log(f"batched {value:.3f} products/s ({step_ms:.1f} ms per step of {args.batch}); max abs error {err:.2e}")

    # the same batched step captured once into a HIP graph and replayed (no host launch work)
    # the same batched step captured once into a HIP graph and replayed (no host launch work);
    # run after the other legs: once a graph has run on the context stream, later work there
    # no longer overlapped the side stream in our measurements (the mixed batch lost its gain)
    def graph_leg():
        log("graph capture of the batched step")
        g, gouts = ctx.matmul_batch_graph(As, Bs, [h] * args.batch)
        ctx.sync()
        same = bool(np.array_equal(ctx.export(gouts[0]), ctx.export(out[0])))
        g.launch()
        ctx.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            g.launch()
        ctx.sync()
        torch.cuda.synchronize()
        gdt = (time.perf_counter() - t0) / args.steps
        res = {"matmuls_per_s": round(args.batch / gdt, 3), "ms_per_step": round(gdt * 1e3, 2),
               "over_eager": round(step_ms / (gdt * 1e3), 3), "bit_identical_to_eager": same, **g.info()}
        log(f"graph replay {gdt * 1e3:.1f} ms per step ({res['matmuls_per_s']} products/s), identical {same}")
        g.close()
        return res

    # serving: Poisson arrivals of h=64 products at a fraction of the batched capacity
    serve = None
    if args.serve_requests > 0:
        rate = args.serve_load * value
        arrivals = I.poisson_arrivals(5, rate, args.serve_requests)
        log(f"serving {args.serve_requests} requests at {rate:.1f}/s")
        srv = he.Server(ctx, max_batch=args.batch, min_batch=args.serve_min_batch,
                        max_wait_us=int(args.serve_max_wait_ms * 1e3))
        tickets, late = [], {}
        t_start = time.perf_counter()
        for i, ta in enumerate(arrivals):
            while time.perf_counter() - t_start < ta:
                time.sleep(0.0005)
            tk = srv.submit(he.REQ_MATMUL, As[i % args.batch], Bs[i % args.batch], h=h)
            late[tk] = (time.perf_counter() - t_start) - ta  # submit delay counts as queueing
            tickets.append(tk)
        lat, t_last = {}, None
        while len(lat) < len(tickets):
            for tk in tickets:
                if tk not in lat:
                    r = srv.poll(tk)
                    if r is not None:
                        lat[tk] = r[1] + late[tk]  # scheduled arrival -> result on the host
                        t_last = time.perf_counter()
            time.sleep(0.0005)
        srv.stop()
        lats = np.array(list(lat.values()))
        serve = {"requests": len(tickets), "arrival_rate_per_s": round(rate, 2),
                 "served_per_s": round(len(tickets) / (t_last - t_start), 3),
                 "p50_ms": round(float(np.percentile(lats, 50)) * 1e3, 1),
                 "p99_ms": round(float(np.percentile(lats, 99)) * 1e3, 1),
                 "max_batch": args.batch, "min_batch": args.serve_min_batch,
                 "max_wait_ms": args.serve_max_wait_ms}
        log(f"serve p50 {serve['p50_ms']} ms p99 {serve['p99_ms']} ms, {serve['served_per_s']} /s")

    # the other schedules, one batch each, timed without launch events
    others = {}
    if not args.no_other:
        pairs = [I.matrix_pair(1000 + i, h) for i in range(args.batch)]
        for name, flags in SCHEDULES.items():
            if flags == sched:
                continue
            ctx2 = he.Context(prm, h_list=[h], stream=stream.cuda_stream, schedule=flags)
            As2 = [ctx2.encrypt(p[0].ravel(), level=level, nonce=2 * i) for i, p in enumerate(pairs)]
            Bs2 = [ctx2.encrypt(p[1].ravel(), level=level, nonce=2 * i + 1) for i, p in enumerate(pairs)]
            ctx2.matmul_batch(As2, Bs2, [h] * args.batch)
            ctx2.sync()
            t0 = time.perf_counter()
            ctx2.matmul_batch(As2, Bs2, [h] * args.batch)
            ctx2.sync()
            others[name] = round(args.batch / (time.perf_counter() - t0), 4)
            log(f"schedule '{name}': {others[name]:.3f} products/s")
            del As2, Bs2
            ctx2.close()

    # the dominant kernel, timed over the timed region, against the roof that binds it: HBM
    # for every kernel whose algorithmic bytes at 8 TB/s take longer than its arithmetic (a
    # transform pass is ALU-bound only where its butterflies' VALU instructions take longer)
    total_ms = sum(v["ms"] for v in prof_all.values())
    d = prof[dom]
    avg_ms = d["ms"] / max(1, d["launches"])
    nl_ = max(1, d["launches"])
    instr = ((d.get("ops", 0) - d.get("fp_ops", 0)) * BFLY_INSTR + d.get("fp_ops", 0) * FP64_BFLY_INSTR) / nl_
    alu_floor_us = instr / VALU_LANE_OPS * 1e6
    hbm_floor_us = d["bytes"] / nl_ / (HBM_PEAK_GBS * 1e9) * 1e6
    if dom in NTT_KERNELS and alu_floor_us > hbm_floor_us:
        achieved = instr / (avg_ms * 1e-3) / 1e12
        peak = VALU_LANE_OPS / 1e12
        roofline = {"bound": "alu", "achieved": round(achieved, 2), "peak": round(peak, 2),
                    "unit": "T VALU lane-instructions/s (butterflies)", "frac": round(achieved / peak, 4),
                    "traffic": measured_traffic(dom) if args.batch == 16 else None}
    else:
        achieved = d["bytes"] / max(1, d["launches"]) / (avg_ms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": measured_traffic(dom) if args.batch == 16 else None}
    if dom in NTT_KERNELS:
        roofline.update({"hbm_floor_us": round(hbm_floor_us, 2), "alu_floor_us": round(alu_floor_us, 2),
                         "butterflies_per_launch": round(d["ops"] / nl_),
                         "fp64_share": round(d.get("fp_ops", 0) / max(1.0, d["ops"]), 3)})
    roofline.update({"kernel": dom, "algorithmic_bytes_per_launch": round(d["bytes"] / nl_),
                     "avg_launch_us": round(avg_ms * 1e3, 2), "launches": d["launches"],
                     "steps_with_events": args.steps - ev_from,
                     "share_of_gpu_time": round(prof_all[dom]["ms"] / total_ms, 3),
                     "gpu_busy": round(total_ms / (prof_elapsed * 1e3), 3)})
    probe = None
    if not args.no_probe:
        probe = hbm_probe(torch, ctx)
        log(f"hbm probe: {probe}")
        if roofline["bound"] == "hbm":
            best = max(probe["copy_GB/s"], probe["two_reads_one_write_GB/s"])
            roofline["frac_of_achievable"] = round(achieved / best, 4)
            roofline["achievable_GB/s"] = best
    prof = prof_all
    ntt_ms = sum(prof[k]["ms"] for k in NTT_KERNELS)
    ntt_ops = sum(prof[k]["ops"] for k in NTT_KERNELS)
    ntt_fp = sum(prof[k].get("fp_ops", 0) for k in NTT_KERNELS)
    ntt_bytes = sum(prof[k]["bytes"] for k in NTT_KERNELS)
    ntt_instr = (ntt_ops - ntt_fp) * BFLY_INSTR + ntt_fp * FP64_BFLY_INSTR
    ntt_rate = ntt_ops / (ntt_ms * 1e-3) / 1e9
    hbm = {k: round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1) for k, v in prof.items()
           if k not in NTT_KERNELS and v["ms"] > 0}
    step_bytes = sum(v["bytes"] for v in prof.values())

    result = {
        "metric": METRIC, "value": round(value, 4), "unit": "HE-matmuls/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(step_ms, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "C3: batch of packed ct x ct h=64 products (Alg. 3 + App. B), N=2^15, "
                               "Q=60+13x45 bits, P=3x60+56 bits, dnum=3, scale 2^45, inputs at level 13",
                   "batch": args.batch, "h": h, "log_n": 15,
                   "schedule": f"{args.schedule}: {SCHEDULE_TEXT[sched]}",
                   "plain_matmuls_per_s": None if plain_s != plain_s else round(1.0 / plain_s, 4),
                   "plain_ms": None if plain_s != plain_s else round(plain_s * 1e3, 2),
                   "batched_matmuls_per_s_other_schedules": others or None,
                   "batched_over_plain": None if plain_s != plain_s else round(value * plain_s, 3),
                   "max_abs_error": err,
                   "autotune": tune,
                   "graph_replay": None},
        "serve": serve,
        "roofline": roofline,
        "ntt_all_passes": {"achieved": round(ntt_rate, 1), "unit": "Gbutterfly/s",
                           "share_of_gpu_time": round(ntt_ms / total_ms, 3),
                           "fp64_share": round(ntt_fp / max(1.0, ntt_ops), 3),
                           "butterfly_valu_frac": round(ntt_instr / (ntt_ms * 1e-3) / VALU_LANE_OPS, 4),
                           "algorithmic_GB/s": round(ntt_bytes / (ntt_ms * 1e-3) / 1e9, 1),
                           "note": "butterfly_valu_frac: the butterflies' VALU instructions (28 per 64-bit integer "
                                   "butterfly of a 60-bit prime, 8 per FP64 butterfly of a prime below 2^46) over "
                                   "the VALU rate of 39.32 T lane-instructions/s"},
        "hbm_probe": probe,
        "step_traffic": {"algorithmic_GB": round(step_bytes / 1e9, 2),
                         "per_product_GB": round(step_bytes / args.batch / 1e9, 3),
                         "hbm_frac": round(step_bytes / (step_ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
                         "note": "every launch's algorithmic bytes (its operands read once, its results "
                                 "written once) summed over one step, over the timed step time at 8 TB/s"},
        "kernels_note": "one untimed step with every launch timed by HIP events",
        "kernels": {k: {"launches": v["launches"], "ms": round(v["ms"], 3),
                        **({"GB/s": hbm[k]} if k in hbm else {})} for k, v in prof.items()},
    }
    # the other legs make contexts of their own: the headline context gives its cached device
    # blocks back first (it keeps its keys and inputs)
    ctx.pool_limit(1)
    ctx.pool_limit(0)
    if not args.no_shapes:
        log("packed (iota_4), rectangular (16 x 64) and transposition legs")
        result["shapes"] = shapes_leg(he, I, prm, sched, stream, args.batch)
        log(f"shapes: {result['shapes']}")
    if args.mix > 0:
        log(f"mixed batch of {args.mix} (h in 16/32/64, levels 3..13)")
        result["mixed_batch"] = mixed_leg(he, I, prm, sched, stream, args.mix)
        log(f"mixed batch: {result['mixed_batch']}")
    if args.c4 > 0:
        log(f"N=2^16 ReLU + h=32 leg ({args.c4} ciphertexts)")
        result["c4_relu_then_matmul"] = c4_leg(he, I, sched, stream, args.c4)
        log(f"c4: {result['c4_relu_then_matmul']}")
    if args.serve_rings > 0:
        log(f"serving across rings ({args.serve_rings} mixed requests)")
        result["serve_mixed_rings"] = serve_rings_leg(he, I, sched, args.serve_rings, args.serve_load)
        log(f"serve across rings: {result['serve_mixed_rings']}")
    if not args.no_graph:
        result["config"]["graph_replay"] = graph_leg()
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        result["cpu_baseline"] = cpu_baseline(prm, sched)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
