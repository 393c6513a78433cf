#!/usr/bin/env python
"""Throughput of the nonuniform fast Hankel transform on one MI355X.

Workload (one step): the transform g_j = sum_k c_k J_nu(omega_j r_k) at
n = m = 1e6, r ~ U[0,1) unsorted, omega ~ U[0,1e5), c ~ N(0,1), eps = 1e-12,
FP64, for each order nu in {0, 1, 10} (inputs drawn with seeds 2, 3, 4).  Each
transform is planned (device sort, staircase, Alg. 1; on a side stream, so a
plan overlaps the previous transform's execution) and executed on the main
stream; inputs are resident in GPU memory before the timed region.  value =
(n+m) per second over the whole step (3 transforms), timed with the device
synchronised on both sides.

Also reported: execute-only throughput (plans reused), per-stage times from
HIP events recorded on the transform's stream inside the timed region, the
roofline of the dominant kernel, and the CPU oracle (direct O(nm) sum) timed
on a bounded sample of the same workload.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

ORDERS = (0, 1, 10)
DOMINANT_STAGES = ("spread", "rows_asymptotic")    # the candidates for the dominant kernel
SEEDS = {0: 2, 1: 3, 10: 4}
EPS = 1e-12
N = M_OUT = 1_000_000
PEAK_FP64 = 78.6e12          # MI355X FP64 vector, flop/s
PEAK_HBM = 8.0e12            # bytes/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def read_traffic(kernel):
    """HBM bytes per launch of `kernel` (for the spreading stage, its two
    kernels together) from FETCH_SIZE and WRITE_SIZE counters scaled by a
    plain copy of known size, read from the committed counter summary if it
    was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_traffic_large_uniform.txt")
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith((" ", "#")):
                k, v = line.split(":", 1)
                rec[k.strip()] = v.strip()
    if rec.get("sources_sha256") != sources_sha256():
        return None
    fetch, write = float(rec["fetch_bytes_per_launch"]), float(rec["write_bytes_per_launch"])
    return dict(fetch_bytes=fetch, write_bytes=write, bytes=fetch + write,
                source=os.path.relpath(path, ROOT))


def read_step_traffic():
    """HBM bytes of one whole step (every kernel of the three plans and
    executions) from FETCH_SIZE and WRITE_SIZE counters scaled by a plain copy
    of known size, read from the committed counter summary if it was taken
    on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "step_traffic_large_uniform.txt")
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith((" ", "#")):
                k, v = line.split(":", 1)
                rec[k.strip()] = v.strip()
    if rec.get("sources_sha256") != sources_sha256():
        return None
    return dict(bytes_per_step=float(rec["bytes_per_step"]), fetch_bytes_per_step=float(rec["fetch_bytes_per_step"]),
                write_bytes_per_step=float(rec["write_bytes_per_step"]), source=os.path.relpath(path, ROOT))


def sources_sha256():
    """Digest of the HIP sources and headers the kernels are built from."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2411_09583_amd", "csrc")
    for d, names in ((csrc, sorted(os.listdir(csrc))), (os.path.join(ROOT, "include"), ["nuht.h"])):
        for name in names:
            if name.endswith((".hip", ".h")):
                with open(os.path.join(d, name), "rb") as f:
                    h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def copy_calibration():
    import torch
    x = torch.ones(64 * 1024 * 1024 // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": x.numel() * 8, "copies": 3}), flush=True)


class StageProfile:
    """Per-stage times of profiled executions, read from each plan once its
    execution is a step behind (its events have completed by then, so the
    read does not stall the pipeline) and the plan released: at most a step's
    worth of plans stays alive.  stages: the stages to time (events only at
    their boundaries), all by default."""

    def __init__(self, nuht, stages=None):
        import collections
        self.pending = collections.deque()
        self.stages = stages
        self.total = {s: 0.0 for s in nuht.STAGES}
        self.calls = 0
        self.infos = {}

    def add(self, nu, p):
        self.pending.append((nu, p))
        self.drain(len(ORDERS))

    def drain(self, keep=0):
        while len(self.pending) > keep:
            nu, p = self.pending.popleft()
            st, nc = p.profile_read()
            for k, v in st.items():
                self.total[k] += v
            self.calls += nc
            self.infos.setdefault(nu, p.info())
            p.close()


def make_step(torch, nuht, inputs, side, eps, **opts):
    """One step: the three transforms, each planned on the side stream (so its
    sort and subdivision overlap the previous transform's execution) and
    executed on the current stream.  prof: a StageProfile taking the plans
    with stage profiling on, or None (plans released once their execution is
    queued)."""
    def step(prof=None):
        outs = {}
        for nu in ORDERS:
            r, w, c = inputs[nu]
            with torch.cuda.stream(side):
                p = nuht.Plan(r, w, nu, eps, **opts)
            if prof is not None:
                p.profile(True, stages=prof.stages)
            outs[nu] = p.execute(c)
            if prof is not None:
                prof.add(nu, p)
            else:
                p.close()
        return outs
    return step


def bench_loose(torch, nuht, inputs, side, steps=5, warmup=2):
    """The same three transforms at eps = 1e-6, in FP64 and with FP32
    spreading, timed like the headline (plans on the side stream overlapping
    the executions): plan + execute throughput, (n+m)/s."""
    res = {}
    for mode, prec in (("fp64", nuht.NUHT_FP64), ("fp32_spread", nuht.NUHT_FP32_SPREAD)):
        step = make_step(torch, nuht, inputs, side, 1e-6, precision=prec)
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(steps):
            outs = step()
        torch.cuda.synchronize()
        t = (time.perf_counter() - a) / steps
        res[mode] = dict(ms_per_step=1e3 * t, value=len(ORDERS) * (N + M_OUT) / t, _outs=outs)
    log("eps 1e-6:", {k: {kk: vv for kk, vv in v.items() if kk != "_outs"} for k, v in res.items()})
    return res


def sampled_error(g_dev, ref, idx):
    """Relative l2 and normwise max error of the GPU output at the sampled
    outputs idx against the oracle's values ref there."""
    g = g_dev.cpu().numpy()[idx]
    return dict(rel_l2=float(np.linalg.norm(g - ref) / np.linalg.norm(ref)),
                rel_max=float(np.max(np.abs(g - ref)) / np.max(np.abs(ref))))


def host_cpu():
    """The host's CPU model and the cores this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return dict(model=model, logical_cpus=os.cpu_count(), usable_cpus=len(os.sched_getaffinity(0)))


def bench_batched(torch, nuht, workloads, dev, oracle=None):
    """256 independent transforms (nu ~ U{0..63}, n and m log-uniform in
    [1e3, 1e6], omega ~ U[0, n_i), eps = 1e-12): a loop of plan + execute per
    transform on one stream against one nuht_plan_many and graph replays of
    nuht_execute_many."""
    tr = workloads.batch(count=256, seed=5)
    rs = [torch.as_tensor(t["r"], device=dev) for t in tr]
    ws = [torch.as_tensor(t["w"], device=dev) for t in tr]
    cs = [torch.as_tensor(t["c"], device=dev) for t in tr]
    nus = [t["nu"] for t in tr]
    total = sum(t["r"].size + t["w"].size for t in tr)
    torch.cuda.synchronize()
    log(f"batched: {len(tr)} transforms, sum(n+m) = {total:.3e}")

    def looped():
        outs = []
        for r, w, c, nu in zip(rs, ws, cs, nus):
            p = nuht.Plan(r, w, nu, EPS)
            outs.append(p.execute(c))
            p.close()
        return outs

    looped()                                   # warm-up (allocator pools, code objects)
    torch.cuda.synchronize()
    a = time.perf_counter()
    outs_loop = looped()
    torch.cuda.synchronize()
    t_loop = time.perf_counter() - a
    # execute-only loop with the plans kept
    plans = [nuht.Plan(r, w, nu, EPS) for r, w, nu in zip(rs, ws, nus)]
    torch.cuda.synchronize()
    a = time.perf_counter()
    for p, c in zip(plans, cs):
        p.execute(c)
    torch.cuda.synchronize()
    t_loop_exec = time.perf_counter() - a
    for p in plans:
        p.close()
    del plans
    a = time.perf_counter()
    b = nuht.Batch(rs, ws, nus, EPS)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - a
    gs = [torch.empty(w.numel(), dtype=torch.float64, device=dev) for w in ws]
    b.execute(cs, gs)                          # first call captures the graph
    torch.cuda.synchronize()
    reps = 5
    a = time.perf_counter()
    for _ in range(reps):
        b.execute(cs, gs)
    torch.cuda.synchronize()
    t_exec = (time.perf_counter() - a) / reps
    same = all(torch.equal(x, y) for x, y in zip(gs, outs_loop))
    b.close()
    acc = None
    if oracle is not None:
        rng = np.random.default_rng(8)
        worst = dict(rel_l2=0.0, rel_max=0.0)
        a = time.perf_counter()
        for t, g in zip(tr, gs):
            i = rng.choice(t["w"].size, min(16, t["w"].size), replace=False)
            e = sampled_error(g, oracle.dht(t["nu"], t["r"], t["c"], t["w"][i]), i)
            worst = {k: max(worst[k], e[k]) for k in worst}
        acc = dict(sampled_outputs_per_transform=16, worst_rel_l2=worst["rel_l2"], worst_rel_max=worst["rel_max"],
                   oracle_s=time.perf_counter() - a)
    res = dict(transforms=len(tr), sum_n_plus_m=total,
               looped_ms=1e3 * t_loop, looped_execute_ms=1e3 * t_loop_exec,
               batched_plan_ms=1e3 * t_plan, batched_execute_ms=1e3 * t_exec,
               batched_ms=1e3 * (t_plan + t_exec),
               speedup_plan_and_execute=t_loop / (t_plan + t_exec),
               speedup_execute=t_loop_exec / t_exec,
               batched_rate=total / (t_plan + t_exec), batched_execute_rate=total / t_exec,
               identical_to_looped=bool(same), accuracy=acc)
    log("batched:", json.dumps(res))
    return res


def bench_fwd_bwd(torch, nuht, workloads, dev):
    """n = m = 1e6, nu = 5, loss 0.5 |g - y|^2: forward plus the gradient in c,
    r and omega (one plan; orders 4, 5, 6 on its sorted geometry) against six
    independent transforms (forward and transposed at nu, transposed and
    forward at nu -+ 1), each planned on its own."""
    r, w, c, y = (torch.as_tensor(a, device=dev) for a in workloads.differentiation(seed=6))
    nu = 5
    torch.cuda.synchronize()

    def fused():
        p = nuht.Plan(r, w, nu, EPS)
        g = p.execute(c)
        grads = p.gradient(c, g - y)
        return p, grads

    p, _ = fused()                               # warm-up
    p.close()
    torch.cuda.synchronize()
    a = time.perf_counter()
    p, _ = fused()
    torch.cuda.synchronize()
    t_cold = time.perf_counter() - a
    reps = 3
    a = time.perf_counter()
    for _ in range(reps):
        g = p.execute(c)
        p.gradient(c, g - y)
    torch.cuda.synchronize()
    t_warm = (time.perf_counter() - a) / reps
    p.close()

    def independent():
        gbar = None
        for order, transposed, scale in ((nu, False, None), (nu, True, None), (nu - 1, True, "w"),
                                         (nu + 1, True, "w"), (nu - 1, False, "r"), (nu + 1, False, "r")):
            q = nuht.Plan(r, w, order, EPS)
            if not transposed:
                out = q.execute(c * r if scale == "r" else c)
                if gbar is None:
                    gbar = out - y
            else:
                out = q.adjoint(gbar * w if scale == "w" else gbar)
            q.close()

    independent()
    torch.cuda.synchronize()
    a = time.perf_counter()
    independent()
    torch.cuda.synchronize()
    t_ind = time.perf_counter() - a
    res = dict(n=r.numel(), m=w.numel(), nu=nu, fused_cold_ms=1e3 * t_cold, fused_warm_ms=1e3 * t_warm,
               independent_ms=1e3 * t_ind, speedup_cold=t_ind / t_cold, speedup_warm=t_ind / t_warm)
    log("fwd+bwd:", json.dumps(res))
    return res


def bench_pn(torch, nuht, workloads, dev, reps=3):
    """The p = O(n) study at n = m = 1e6, nu = 0, eps = 1e-8 (the configuration of
    the paper's runtime figure for this study): Fourier-Bessel points and
    frequencies (scaled zeros of J_0) and the exponentially distributed case
    (the worst case for the partition).  Then the figure's order sweep
    (nu = 10, 100 at eps = 1e-8) and tolerance sweep (eps = 1e-4 ... 1e-15 at
    nu = 0), Fourier-Bessel only.  Plan + execute per transform."""
    n = 1_000_000

    def timed(arrs, nu, eps, **kw):
        r, w, c = (torch.as_tensor(a, device=dev) for a in arrs)
        p = nuht.Plan(r, w, nu, eps, **kw)           # warm-up
        p.execute(c)
        inf = p.info()
        p.close()
        torch.cuda.synchronize()
        t_plan = t_exec = 0.0
        for _ in range(reps):
            a = time.perf_counter()
            p = nuht.Plan(r, w, nu, eps, **kw)
            torch.cuda.synchronize()
            b = time.perf_counter()
            p.execute(c)
            torch.cuda.synchronize()
            e = time.perf_counter()
            p.close()
            t_plan += b - a
            t_exec += e - b
        t_plan /= reps
        t_exec /= reps
        return dict(n=n, m=n, nu=nu, eps=eps, plan_ms=1e3 * t_plan, execute_ms=1e3 * t_exec,
                    value=2 * n / (t_plan + t_exec), execute_rate=2 * n / t_exec, levels=inf["levels"],
                    blocks=[inf["n_local"], inf["n_asy"], inf["n_direct"]], M=inf["M"], L=inf["L"])

    fb0 = workloads.fourier_bessel(n, 0, seed=160)
    res = {"fourier_bessel": timed(fb0, 0, 1e-8),
           "exponential": timed(workloads.exponential(n, seed=161), 0, 1e-8)}
    for kind in ("fourier_bessel", "exponential"):
        log("p=O(n):", kind, json.dumps(res[kind]))
    sweep = []
    for eps in (1e-4, 1e-6, 1e-10, 1e-12, 1e-15):
        sweep.append(timed(fb0, 0, eps))
    tail = []
    for nu in (10, 100):
        fb = workloads.fourier_bessel(n, nu, seed=160 + nu)
        sweep.append(timed(fb, nu, 1e-8))
        tail.append(timed(fb, nu, 1e-8, local_rank=-1))
    keep = ("nu", "eps", "plan_ms", "execute_ms", "value", "M", "L", "levels")
    res["fourier_bessel_sweep"] = [{k: d[k] for k in keep} for d in sweep]
    # the same two orders with the tail-sum local rank (local_rank = -1)
    res["fourier_bessel_tail_rank"] = [{k: d[k] for k in keep} for d in tail]
    for d in res["fourier_bessel_tail_rank"]:
        log("p=O(n): fourier_bessel tail rank", json.dumps(d))
    for d in res["fourier_bessel_sweep"]:
        log("p=O(n): fourier_bessel sweep", json.dumps(d))
    return res


def bench_disk(torch, nuht, workloads, dev, reps=5, method="transform"):
    """The Helmholtz solver on the unit disk (Sec. 5.3) at the paper's example
    kappa = 25, eps = 1e-8: m = 512 Gauss-Legendre radii, t = 256 angles,
    orders -100 .. 100, J = 128 radial modes per order, a random smooth
    forcing.  Solver planning once, then analysis, synthesis and the whole
    solve (analysis, division by the eigenvalues, synthesis), each timed over
    `reps` calls.  With the transform method a solve runs 4 (L + 1) transforms
    (real and imaginary parts per order |l|, both directions; orders -l and l
    share them) of n + m = 512 + 128 each; the direct method takes the same
    sums term by term, 2 (L + 1) m J Bessel evaluations per solve."""
    m, t, L, J, eps, kappa = 512, 256, 100, 128, 1e-8, 25.0
    r, wr, zeros, f = workloads.disk(m, t, L, J, seed=190)
    rd, wrd, zd, fd = (torch.as_tensor(a, device=dev) for a in (r, wr, zeros, f))
    torch.cuda.synchronize()
    a = time.perf_counter()
    s = nuht.DiskSolver(rd, wrd, t, zd, eps, method=method)
    torch.cuda.synchronize()
    plan_ms = 1e3 * (time.perf_counter() - a)
    alpha = s.analysis(fd)
    beta = alpha.clone()
    s.synthesis(beta)
    s.helmholtz(kappa, fd)                       # warm-up of every path
    torch.cuda.synchronize()

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t0) / reps

    an_ms = timed(lambda: s.analysis(fd))
    sy_ms = timed(lambda: s.synthesis(beta))
    he_ms = timed(lambda: s.helmholtz(kappa, fd))
    s.close()
    transforms = 4 * (L + 1)
    res = dict(method=method, m=m, t=t, L=L, J=J, eps=eps, kappa=kappa, plan_ms=plan_ms, analysis_ms=an_ms,
               synthesis_ms=sy_ms, solve_ms=he_ms)
    if method == "transform":
        res.update(transforms_per_solve=transforms, transform_rate=transforms * (m + J) / (he_ms * 1e-3))
    else:
        res.update(bessel_per_solve=2 * (L + 1) * m * J)
    log("disk solver:", json.dumps(res))
    return res


def bench_radial(torch, nuht, workloads, dev, oracle=None, reps=5):
    """The radial 2-D Fourier-transform workload at its full size (n = m = 1e6
    Chebyshev-clustered points, c = r w exp(-40 r^2) cos(30 r), log-spaced
    frequencies on [1e-2, 1e5], nu = 0, eps = 1e-12), the stand-in for the
    study of Sec. 5.2 and the most direct-heavy configuration: plan and
    execute times and (n+m)/s, and the error on 256 sampled outputs."""
    r_np, w_np, c_np = workloads.radial_2d()
    r, w, c = (torch.as_tensor(a, device=dev) for a in (r_np, w_np, c_np))
    p = nuht.Plan(r, w, 0, EPS)
    g = p.execute(c)
    inf = p.info()
    p.close()
    torch.cuda.synchronize()
    t_plan = t_exec = 0.0
    for _ in range(reps):
        a = time.perf_counter()
        p = nuht.Plan(r, w, 0, EPS)
        torch.cuda.synchronize()
        b = time.perf_counter()
        g = p.execute(c)
        torch.cuda.synchronize()
        e = time.perf_counter()
        p.close()
        t_plan += (b - a) / reps
        t_exec += (e - b) / reps
    n = r.numel() + w.numel()
    res = dict(n=r.numel(), m=w.numel(), nu=0, eps=EPS, plan_ms=1e3 * t_plan, execute_ms=1e3 * t_exec,
               value=n / (t_plan + t_exec), execute_rate=n / t_exec, levels=inf["levels"],
               blocks=[inf["n_local"], inf["n_asy"], inf["n_direct"]], direct_entries=inf["direct_entries"])
    if oracle is not None:
        idx = np.random.default_rng(9).choice(w_np.size, 256, replace=False)
        res["accuracy"] = dict(sampled_outputs=256, **sampled_error(g, oracle.dht(0, r_np, c_np, w_np[idx]), idx))
    log("radial 2-D:", json.dumps(res))
    return res


def bench_split(torch, nuht, r, w, c, reps=5):
    """Exact against quasi-optimal SplitIndices (Sec. 4.1) at the large uniform
    workload, nu = 0, eps = 1e-12: plan and execute times and the partition's
    direct area for 16 candidate rows per split (the default) and for every
    row (split_candidates = -1)."""
    res = {}
    for name, cand in (("quasi_16", 0), ("exact", -1)):
        torch.cuda.synchronize()
        a = time.perf_counter()
        p = nuht.Plan(r, w, 0, EPS, split_candidates=cand)
        torch.cuda.synchronize()
        b = time.perf_counter()
        p.execute(c)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            p.execute(c)
        torch.cuda.synchronize()
        ex = 1e3 * (time.perf_counter() - t0) / reps
        inf = p.info()
        p.close()
        res[name] = dict(plan_ms=1e3 * (b - a), execute_ms=ex, levels=inf["levels"],
                         blocks=[inf["n_local"], inf["n_asy"], inf["n_direct"]], direct_entries=inf["direct_entries"],
                         asy_col_members=inf["asy_col_members"], local_row_members=inf["local_row_members"])
    log("split:", json.dumps(res))
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-sample", type=int, default=4096,
                    help="outputs of the nu=0 transform computed by the CPU oracle")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-vs-looped comparison")
    ap.add_argument("--no-grad", action="store_true", help="skip the forward+backward comparison")
    ap.add_argument("--no-loose", action="store_true", help="skip the eps = 1e-6 (FP64 and FP32 spreading) runs")
    ap.add_argument("--no-disk", action="store_true", help="skip the disk Helmholtz solver leg")
    ap.add_argument("--no-split", action="store_true", help="skip the exact-split comparison")
    ap.add_argument("--no-radial", action="store_true", help="skip the radial 2-D workload at n = m = 1e6")
    ap.add_argument("--no-pn", action="store_true",
                    help="skip the p = O(n) study (Fourier-Bessel and exponential points at n = m = 1e6)")
    ap.add_argument("--steps-only", action="store_true",
                    help="only the warmup and timed headline steps (for hardware-counter runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 64 MiB device-to-device copy three times (a known byte count "
                         "for scaling the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return

    import torch
    import paper_2411_09583_amd as nuht
    import workloads

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    nuht.load_library()
    inputs = {}
    for nu in ORDERS:
        r, w, c = workloads.large_uniform(seed=SEEDS[nu], n=N, m=M_OUT)
        inputs[nu] = tuple(torch.as_tensor(a, device=dev) for a in (r, w, c))
    torch.cuda.synchronize()
    log("inputs resident")

    # Plans are made on a side stream (the inputs are resident), so each plan's
    # sort and subdivision overlap the previous transform's execution on the
    # main stream; the plan is complete when Plan() returns.
    side = torch.cuda.Stream()
    step = make_step(torch, nuht, inputs, side, EPS)

    for _ in range(args.warmup):
        step(None)
    torch.cuda.synchronize()
    log("warmup done")

    # Inside the timed region events bracket only the two stages that can be
    # the dominant kernel (the spreading and the asymptotic rows), whose
    # live durations the roofline uses; the other stages are timed in an
    # untimed pass afterwards, so that the timed steps carry few events.
    prof = StageProfile(nuht, stages=DOMINANT_STAGES)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        outs = step(prof)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof.drain()
    elapsed = t1 - t0
    ms_per_step = 1e3 * elapsed / args.steps
    work = len(ORDERS) * (N + M_OUT)
    value = work * args.steps / elapsed
    log(f"timed: {ms_per_step:.3f} ms/step, {value:.4e} (n+m)/s")
    if args.steps_only:
        # for counter runs: the library's kernels of this process are exactly
        # warmup + steps headline steps
        print(json.dumps({"steps_only": True, "warmup": args.warmup, "steps": args.steps,
                          "ms_per_step": ms_per_step, "value": value}), flush=True)
        return

    # per-stage times: the dominant-kernel candidates from events recorded
    # inside the timed region, the others from an untimed pass with every
    # stage profiled
    infos = prof.infos
    live_ms = {k: prof.total[k] / args.steps for k in DOMINANT_STAGES}   # per step (3 transforms)
    prof_all = StageProfile(nuht)
    all_steps = 5
    for _ in range(all_steps):
        step(prof_all)
    torch.cuda.synchronize()
    prof_all.drain()
    stage_ms = {k: v / all_steps for k, v in prof_all.total.items()}
    untimed_ms = dict(stage_ms)
    stage_ms.update(live_ms)

    # execute-only and plan-only times per order
    per_order = {}
    for nu in ORDERS:
        r, w, c = inputs[nu]
        torch.cuda.synchronize()
        a = time.perf_counter()
        p = nuht.Plan(r, w, nu, EPS)
        torch.cuda.synchronize()
        b = time.perf_counter()
        reps = max(3, args.steps)
        for _ in range(reps):
            g = p.execute(c)
        torch.cuda.synchronize()
        e = time.perf_counter()
        inf = p.info()
        p.close()
        ex_ms = 1e3 * (e - b) / reps
        per_order[str(nu)] = dict(plan_ms=1e3 * (b - a), execute_ms=ex_ms,
                                  execute_rate=(N + M_OUT) / (ex_ms * 1e-3),
                                  M=inf["M"], L=inf["L"], z=inf["z"], es_width=inf["es_width"],
                                  levels=inf["levels"], blocks=[inf["n_local"], inf["n_asy"], inf["n_direct"]],
                                  asy_members=[inf["asy_row_members"], inf["asy_col_members"]],
                                  local_members=[inf["local_row_members"], inf["local_col_members"]],
                                  direct_entries=inf["direct_entries"], fft_points=inf["fft_points"])
    exec_total = sum(v["execute_ms"] for v in per_order.values())
    log("per order:", json.dumps(per_order))
    log("stage ms per step:", json.dumps(stage_ms), "(live in the timed steps:", ", ".join(DOMINANT_STAGES),
        "; untimed pass:", json.dumps({k: untimed_ms[k] for k in DOMINANT_STAGES}), ")")

    # Roofline of the dominant kernel among those with an algorithmic flop
    # count (FP64 operations the method's arithmetic needs, per launch; phase
    # evaluations and index arithmetic are not counted):
    #   spreading   (k_spread_mfma on dense items, k_spread on the others; one
    #               stage) every (point, tap) pair inside the kernel support (w taps
    #               per point membership): the kernel value from its degree-13
    #               polynomial piece (13 multiply-adds, 26 flops), then 2M complex
    #               channels x (2 add + 2 mul) and the kernel-weight product:
    #               26 + 8M + 2 (without the kernel evaluation: 8M + 2)
    #   k_rows_asy  every (row, cell) pair of a direct-sum-path block: channel
    #               sum (2M-1) x 4, one complex multiply-add of Horner's rule over
    #               the cells 8: 8M + 4; every (row, tap) pair of an FFT-path
    #               block: (2M-1) x 4 + 4 = 8M, plus the tap's kernel value
    def flops(stage, inf, with_kernel=True):
        M, w = inf["M"], inf["es_width"]
        kv = 26.0 if with_kernel else 0.0
        if stage == "spread":
            return inf["asy_col_members"] * w * (kv + 8.0 * M + 2.0)
        return inf["dft_row_cells"] * (8.0 * M + 4.0) + inf["fft_row_members"] * w * (kv + 8.0 * M)

    kern = {"spread": "k_spread_mfma+k_spread", "rows_asymptotic": "k_rows_asy"}
    tfile = {"spread": "spread_stage", "rows_asymptotic": "k_rows_asy"}   # traffic summaries
    dom = max(kern, key=lambda st: stage_ms[st])
    fl = sum(flops(dom, infos[nu]) for nu in ORDERS)             # one launch per order per step
    fl_ch = sum(flops(dom, infos[nu], False) for nu in ORDERS)
    achieved = fl / (stage_ms[dom] * 1e-3)
    traffic = read_traffic(tfile[dom])
    roofline = dict(bound="alu", kernel=kern[dom], achieved=achieved / 1e12, peak=PEAK_FP64 / 1e12,
                    unit="TFLOP/s", frac=achieved / PEAK_FP64, traffic=traffic,
                    flops_per_step=fl, launches_per_step=len(ORDERS),
                    frac_without_kernel_evaluation=fl_ch / (stage_ms[dom] * 1e-3) / PEAK_FP64,
                    ms_per_step={k: stage_ms[k] for k in kern})
    # In the timed steps the local moments and direct blocks run on the
    # library's side stream beside the spreading chain, so the dominant
    # stage's event-timed duration includes sharing the GPU with them; the
    # untimed pass (every stage timed) runs all stages on one stream, which
    # gives the kernel's own rate.
    one_ms = untimed_ms[dom]
    roofline["one_stream"] = dict(ms_per_step=one_ms, achieved=fl / (one_ms * 1e-3) / 1e12,
                                  frac=fl / (one_ms * 1e-3) / PEAK_FP64)
    if traffic is not None:
        gbs = len(ORDERS) * traffic["bytes"] / (stage_ms[dom] * 1e-3)
        roofline.update(traffic_GBps=gbs / 1e9, hbm_frac=gbs / PEAK_HBM)
    # The other stages with an algorithmic count, each over its own event-timed
    # duration (the asymptotic rows live in the timed steps, the direct blocks
    # and local moments in the untimed profiled pass): the asymptotic rows (as
    # above); the direct
    # blocks at 200 flops per entry (one J_nu(omega r) and its multiply-add,
    # the survey's per-entry estimate; the table evaluation spends ~34); the
    # local moments at 4 (L + 1) flops per local column membership (a
    # Chebyshev step and a multiply-add per moment).
    stage_flops = {
        "spread": fl,
        "rows_asymptotic": sum(flops("rows_asymptotic", infos[nu]) for nu in ORDERS),
        "direct": sum(200.0 * infos[nu]["direct_entries"] for nu in ORDERS),
        "local_moments": sum(4.0 * (infos[nu]["L"] + 1) * infos[nu]["local_col_members"] for nu in ORDERS),
    }
    roofline["stages"] = {
        st: dict(flops_per_step=f, ms_per_step=stage_ms[st], achieved=f / (stage_ms[st] * 1e-3) / 1e12,
                 frac=f / (stage_ms[st] * 1e-3) / PEAK_FP64)
        for st, f in stage_flops.items() if stage_ms[st] > 0}
    step_traffic = read_step_traffic()
    if step_traffic is not None:
        gbs = step_traffic["bytes_per_step"] / (ms_per_step * 1e-3)
        step_traffic.update(GBps=gbs / 1e9, hbm_frac=gbs / PEAK_HBM)
        log("whole-step HBM traffic:", json.dumps(step_traffic))

    loose = None if args.no_loose else bench_loose(torch, nuht, inputs, side)

    # CPU baseline: the oracle's direct sum, on all host cores, for a sample of
    # the nu = 0 outputs (all 1e6 points each), extrapolated to the whole
    # transform, and once more on one thread for a smaller sample.  The oracle
    # values at sampled outputs of every order give the GPU outputs' errors.
    cpu = None
    accuracy = None
    odirect = None
    if not args.no_cpu_baseline:
        from oracle import direct as odirect
        threads = odirect.max_threads()
        samples = {0: args.cpu_sample, 1: 512, 10: 512}
        accuracy = {"eps": EPS, "orders": {}}
        for nu in ORDERS:
            r, w, c = (t.cpu().numpy() for t in inputs[nu])
            k = samples[nu]
            idx = np.random.default_rng(7 + nu).choice(M_OUT, k, replace=False)
            a = time.perf_counter()
            ref = odirect.dht(nu, r, c, w[idx], nthreads=threads)
            b = time.perf_counter()
            if nu == 0:
                full_s = (b - a) * M_OUT / k
                k1 = 64
                a1 = time.perf_counter()
                odirect.dht(0, r, c, w[idx[:k1]], nthreads=1)
                one_s = (time.perf_counter() - a1) * M_OUT / k1
                cpu = dict(value=(N + M_OUT) / full_s, unit="(n+m)/s", cores=threads, kind="oracle",
                           sample=f"direct sum for {k} of the 1e6 outputs (all 1e6 points, nu=0), "
                                  f"{b - a:.1f} s on {threads} threads, extrapolated to the full transform",
                           one_thread=dict(value=(N + M_OUT) / one_s, unit="(n+m)/s",
                                           sample=f"{k1} outputs on 1 thread, extrapolated"),
                           host=host_cpu())
                log("cpu baseline", cpu)
            accuracy["orders"][str(nu)] = dict(sampled_outputs=k, **sampled_error(outs[nu], ref, idx))
            if loose is not None:
                for mode in ("fp64", "fp32_spread"):
                    loose[mode].setdefault("accuracy", {})[str(nu)] = dict(
                        sampled_outputs=k, **sampled_error(loose[mode]["_outs"][nu], ref, idx))
        log("accuracy", accuracy)
    if loose is not None:
        for mode in ("fp64", "fp32_spread"):
            loose[mode].pop("_outs", None)

    batched = None if args.no_batched else bench_batched(torch, nuht, workloads, dev, odirect)
    radial = None if args.no_radial else bench_radial(torch, nuht, workloads, dev, odirect)
    fwd_bwd = None if args.no_grad else bench_fwd_bwd(torch, nuht, workloads, dev)
    pn = None if args.no_pn else bench_pn(torch, nuht, workloads, dev)
    disk = None if args.no_disk else {meth: bench_disk(torch, nuht, workloads, dev, method=meth)
                                      for meth in ("transform", "direct")}
    split = None if args.no_split else bench_split(torch, nuht, *inputs[0])

    out = {
        "metric": "(n+m)/s at eps=1e-12 vs direct sum; batched and fwd+bwd speedup, HBM GB/s",
        "value": value,
        "unit": "(n+m)/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "large uniform: n=m=1e6, r~U[0,1) unsorted, omega~U[0,1e5), c~N(0,1), "
                               "eps=1e-12, one transform each for nu=0,1,10 (plan+execute)",
                   "n": N, "m": M_OUT, "orders": list(ORDERS), "eps": EPS},
        "execute_only_value": len(ORDERS) * (N + M_OUT) / (exec_total * 1e-3),
        "per_order": per_order,
        "stage_ms_per_step": stage_ms,
        "stage_ms_source": {"timed_region": list(DOMINANT_STAGES),
                            "untimed_pass": [k for k in stage_ms if k not in DOMINANT_STAGES]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "accuracy": accuracy,
        "step_traffic": step_traffic,
        "batched": batched,
        "radial_2d": radial,
        "fwd_bwd": fwd_bwd,
        "eps_1e-6": loose,
        "p_equals_n": pn,
        "disk_helmholtz": disk,
        "split_exact": split,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
