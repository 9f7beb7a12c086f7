"""Autotuner: exhaustive timing of kernel configurations per problem shape.

The paper picks its number of groups G by sampling a few HSUMMA iterations
with different values (Sec. V-A's model validation, Sec. VI).  On one GPU the
knobs that change speed but not the product are the kernel configuration of
the local update: the macro-tile, k-chunk and waves per workgroup of the
FP64 path, the grouped persistent launch, and the precision form (the split
forms with their per-panel slice count, which the library chooses to meet
the FP64 accuracy target and replaces by the FP64 kernel on panels it cannot
carry, so every candidate is FP64-accurate).  The tuner times one outer step
(hsumma_outer_update: every inner step of one outer block, one launch) of
each candidate -- per-step cost is uniform over the steps -- and keeps the
fastest.  The inner block b does not enter: within an outer update the
kernels only restart their 4-deep MFMA k-groups at inner-step boundaries
(`b_axis` measures it); b matters to callers that launch every inner step
on its own (hsumma_local_update), where a larger b means fewer C round trips.

Results are cached as JSON (path from $HSUMMA_TUNE_CACHE or an argument),
keyed by the shape.
"""
from __future__ import annotations

import json
import math
import os
import time
from dataclasses import asdict, dataclass

from . import hsumma as hs

# (name, plan options).  FP64 tiles are the configurations compiled into the
# library; the split form picks its slice count per panel.
CANDIDATES = [
    ("fp64_128x128x16", dict(prec=hs.FP64, tile_m=128, tile_n=128, kc=16)),
    ("fp64_128x128x8", dict(prec=hs.FP64, tile_m=128, tile_n=128, kc=8)),
    ("fp64_128x128x32", dict(prec=hs.FP64, tile_m=128, tile_n=128, kc=32)),
    ("fp64_256x128x8", dict(prec=hs.FP64, tile_m=256, tile_n=128, kc=8)),
    ("fp64_256x128x16", dict(prec=hs.FP64, tile_m=256, tile_n=128, kc=16)),
    ("fp64_128x64x16", dict(prec=hs.FP64, tile_m=128, tile_n=64, kc=16)),
    ("fp64_64x128x16", dict(prec=hs.FP64, tile_m=64, tile_n=128, kc=16)),
    ("fp64_64x64x16", dict(prec=hs.FP64, tile_m=64, tile_n=64, kc=16)),
    ("fp64_64x64x32", dict(prec=hs.FP64, tile_m=64, tile_n=64, kc=32)),
    ("fp64_32x32x16", dict(prec=hs.FP64, tile_m=32, tile_n=32, kc=16)),
    ("fp64_128x128x16_w8", dict(prec=hs.FP64, tile_m=128, tile_n=128, kc=16, waves=8)),
    ("fp64_128x256x16", dict(prec=hs.FP64, tile_m=128, tile_n=256, kc=16)),
    ("fp64_64x256x16", dict(prec=hs.FP64, tile_m=64, tile_n=256, kc=16)),
    ("fp64_256x64x16", dict(prec=hs.FP64, tile_m=256, tile_n=64, kc=16)),
    ("fp64_128x128x16_persistent", dict(prec=hs.FP64, tile_m=128, tile_n=128, kc=16,
                                        persistent=1)),
    ("fp64_64x64x16_persistent", dict(prec=hs.FP64, tile_m=64, tile_n=64, kc=16, persistent=1)),
    ("split_bf16", dict(prec=hs.SPLIT_BF16)),
    ("split_int8", dict(prec=hs.SPLIT_INT8)),
]
NAMES = [c[0] for c in CANDIDATES]
DEFAULT = "fp64_128x128x16"   # the fixed configuration the regret reports compare against
SPLIT_MAX_SIGMA = 2.0         # spread up to which the splits carry every panel (a feature)


def library_default(shape) -> str:
    """The configuration the library picks without tuning (hsumma_plan with
    no tile options), as the plan reports it."""
    s = shape if isinstance(shape, dict) else shape.__dict__
    p = hs.Plan(s["n"], s["P"], s["Q"], s["G"], s["M"], s["M"], m=s["m"], k=s["k"])
    tm, tn, kc, _ = p.tile_config
    p.close()
    return "fp64_%dx%dx%d" % (tm, tn, kc)


@dataclass(frozen=True)
class Shape:
    m: int
    n: int
    k: int
    P: int
    Q: int
    G: int
    M: int
    sigma: float = 0.0

    def key(self) -> str:
        return "m%d_n%d_k%d_P%d_Q%d_G%d_M%d_s%g" % (self.m, self.n, self.k, self.P, self.Q,
                                                    self.G, self.M, self.sigma)


def allowed(shape: Shape, name: str) -> bool:
    # every candidate computes an FP64-accurate product: the split forms send
    # the panels their slice-count model cannot carry to the FP64 kernel
    return name in NAMES


def operands(shape: Shape, seed: int = 0):
    """Device operands of the shape's distribution (generated on the GPU)."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)

    def draw(r, c):
        u = torch.rand((r, c), dtype=torch.float64, device="cuda", generator=g) * 2 - 1
        if shape.sigma > 0:
            e = torch.round(torch.randn((r, c), dtype=torch.float64, device="cuda", generator=g)
                            * shape.sigma)
            u = torch.ldexp(u, e.to(torch.int32))
        return u

    A = draw(shape.m, shape.k)
    B = draw(shape.k, shape.n)
    C = torch.zeros((shape.m, shape.n), dtype=torch.float64, device="cuda")
    return A, B, C


def time_candidate(shape: Shape, opts: dict, A, B, C, reps: int = 3) -> float:
    """Median time (ms) of one outer step with the given options."""
    import torch
    plan = hs.Plan(shape.n, shape.P, shape.Q, shape.G, shape.M, shape.M, m=shape.m, k=shape.k,
                   **opts)
    ws = plan.workspace()
    stream = torch.cuda.current_stream()
    plan.outer_update(0, A, B, C, ws=ws)          # warm-up
    times = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        plan.outer_update(0, A, B, C, ws=ws)
        e1.record(stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    plan.close()
    times.sort()
    return times[len(times) // 2]


def time_shape(shape: Shape, names=None, reps: int = 3, seed: int = 0) -> dict:
    """{candidate name: ms} for every allowed candidate."""
    A, B, C = operands(shape, seed)
    out = {}
    for name, opts in CANDIDATES:
        if names is not None and name not in names:
            continue
        if not allowed(shape, name):
            continue
        out[name] = time_candidate(shape, opts, A, B, C, reps)
    del A, B, C
    return out


def best(times: dict) -> str:
    return min(times, key=times.get)


class Cache:
    """JSON cache: shape key -> {"times": {...}, "best": name}."""

    def __init__(self, path: str | None = None):
        self.path = path or os.environ.get("HSUMMA_TUNE_CACHE", "")
        self.data = {}
        if self.path and os.path.exists(self.path):
            with open(self.path) as f:
                self.data = json.load(f)

    def get(self, shape: Shape):
        return self.data.get(shape.key())

    def put(self, shape: Shape, times: dict):
        self.data[shape.key()] = {"shape": asdict(shape), "times": times, "best": best(times)}

    def save(self):
        if self.path:
            tmp = self.path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.data, f)
            os.replace(tmp, self.path)


def tune(shape: Shape, cache: Cache | None = None, reps: int = 3) -> tuple[str, dict]:
    """Exhaustive search: (best candidate name, plan options), cached."""
    cache = cache if cache is not None else Cache()
    hit = cache.get(shape)
    if hit is None:
        times = time_shape(shape, reps=reps)
        cache.put(shape, times)
        cache.save()
        hit = cache.get(shape)
    name = hit["best"]
    return name, dict(CANDIDATES)[name]


def b_axis(n: int = 4096, P: int = 4, Q: int = 4, G: int = 4, M: int = 512,
           bs=(32, 64, 128, 256, 512), reps: int = 5) -> dict:
    """Time of one outer update (ms) and of the same k-range as separate
    local updates (ms per outer block) for each inner block b | M, FP64."""
    import torch
    sh = Shape(n, n, n, P, Q, G, M)
    A, B, C = operands(sh, 1306)
    stream = torch.cuda.current_stream()
    out = {}
    for b in bs:
        if b > M or M % b:
            continue
        plan = hs.Plan(n, P, Q, G, b, M)
        ws = plan.workspace()
        steps = M // b

        def outer():
            plan.outer_update(0, A, B, C, ws=ws)

        def local():
            for s in range(steps):
                plan.local_update(s, A, B, C, ws=ws)
        res = {}
        for nm, fn in (("outer_ms", outer), ("local_ms", local)):
            fn()
            ts = []
            for _ in range(reps):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                fn()
                e1.record(stream)
                e1.synchronize()
                ts.append(e0.elapsed_time(e1))
            res[nm] = sorted(ts)[len(ts) // 2]
        out[b] = res
        plan.close()
    return out


def valid_groups(P: int, Q: int) -> list[int]:
    """Every G that can be arranged as I x J groups with I | P and J | Q."""
    out = set()
    for I in range(1, P + 1):
        if P % I:
            continue
        for J in range(1, Q + 1):
            if Q % J == 0:
                out.add(I * J)
    return sorted(out)


def random_shapes(count: int, seed: int, lo: int = 512, hi: int = 16384):
    """Random problem shapes: m, n, k log-uniform in [lo, hi], P, Q in 1..16,
    G uniform over the arrangeable group counts, outer block M in
    {32, ..., 512}, exponent spread sigma in {0, 2, 4}."""
    import numpy as np
    r = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        m, n, k = (int(round(math.exp(r.uniform(math.log(lo), math.log(hi))))) for _ in range(3))
        P, Q = int(r.integers(1, 17)), int(r.integers(1, 17))
        G = int(r.choice(valid_groups(P, Q)))
        M = int(r.choice([32, 64, 128, 256, 512]))
        sigma = float(r.choice([0.0, 2.0, 4.0]))
        out.append(Shape(m, n, k, P, Q, G, min(M, k), sigma))
    return out


def build_dataset(shapes, reps: int = 3, log=None) -> list:
    """Time every allowed candidate of every shape: [{"shape", "times"}]."""
    rows = []
    t0 = time.time()
    for i, sh in enumerate(shapes):
        rows.append({"shape": asdict(sh), "times": time_shape(sh, reps=reps, seed=i)})
        if log and (i + 1) % 50 == 0:
            log("timed %d/%d shapes (%.0f s)" % (i + 1, len(shapes), time.time() - t0))
    return rows


# -- the number of groups G: by the cost model and by sampling ---------------
# The paper chooses G by sampling a few HSUMMA iterations with the valid
# values (Sec. V-A2, Sec. VI); its model (Sec. IV) says whether G = sqrt(p)
# beats SUMMA on a platform of latency alpha and reciprocal bandwidth beta.
# On one GPU G changes no communication, only the order of the work items
# (group by group, each group's tiles sharing an XCD's L2), so the sampled
# times measure that effect alone.

PLATFORMS = {   # the paper's parameter sets (Sec. V), seconds and seconds per element
    "grid5000": dict(alpha=1e-4, beta=1e-9),
    "bgp": dict(alpha=3e-6, beta=1e-9),
    "exascale": dict(alpha=5e-7, beta=1e-11),
}


def group_counts(P: int, Q: int) -> list[int]:
    return valid_groups(P, Q)


def select_groups_by_model(n: int, P: int, Q: int, b: int, B: int, alpha: float, beta: float,
                           algo: int = hs.BCAST_VAN_DE_GEIJN) -> dict:
    G, best, summa = hs.model_select_groups(algo, alpha, beta, 0.0, n, P, Q, b, B)
    return {"G": G, "comm_s": best["comm"], "summa_comm_s": summa["comm"],
            "ratio": summa["comm"] / best["comm"] if best["comm"] > 0 else 1.0,
            "sqrt_p_is_minimum": alpha / beta > 2.0 * n * b / (P * Q)}


def select_groups_by_sampling(n: int, P: int, Q: int, b: int, M: int, counts=None,
                              steps: int = 2, reps: int = 3, prec=hs.FP64) -> dict:
    """Time `steps` outer steps of HSUMMA for every G (median of `reps`) and
    keep the fastest: {"G": best, "ms": {G: ms per outer step}}."""
    import torch
    counts = counts or group_counts(P, Q)
    g = torch.Generator(device="cuda")
    g.manual_seed(4161)
    A = torch.rand((n, n), dtype=torch.float64, device="cuda", generator=g) * 2 - 1
    B = torch.rand((n, n), dtype=torch.float64, device="cuda", generator=g) * 2 - 1
    C = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    plans = {G: hs.Plan(n, P, Q, G, b, M, prec=prec) for G in counts}
    wss = {G: plans[G].workspace() for G in counts}
    nsteps = min(steps, plans[counts[0]].num_outer_steps)

    def run(G):
        for s in range(nsteps):
            plans[G].outer_update(s, A, B, C, ws=wss[G])
    for G in counts:                        # warm-up: clocks up
        run(G)
    torch.cuda.synchronize()
    # the counts take turns in every repetition, so that clock or thermal
    # drift during the sampling falls on all of them alike
    times = {G: [] for G in counts}
    for _ in range(reps):
        for G in counts:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            run(G)
            e1.record(stream)
            e1.synchronize()
            times[G].append(e0.elapsed_time(e1) / nsteps)
    for G in counts:
        plans[G].close()
    del A, B, C, wss
    out = {G: sorted(v)[len(v) // 2] for G, v in times.items()}
    return {"G": min(out, key=out.get), "ms": out}


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser(prog="python -m paper_1306_4161_amd.tune")
    sub = ap.add_subparsers(dest="cmd", required=True)
    gp = sub.add_parser("groups", help="choose G by the cost model and by sampling")
    gp.add_argument("--n", type=int, default=8192)
    gp.add_argument("--P", type=int, default=8)
    gp.add_argument("--Q", type=int, default=8)
    gp.add_argument("--b", type=int, default=64)
    gp.add_argument("--M", type=int, default=256)
    gp.add_argument("--steps", type=int, default=2)
    gp.add_argument("--no-sample", action="store_true", help="model only (no GPU)")
    bp = sub.add_parser("baxis", help="outer vs local update time over the inner block b")
    bp.add_argument("--n", type=int, default=4096)
    bp.add_argument("--M", type=int, default=512)
    args = ap.parse_args(argv)
    if args.cmd == "baxis":
        print(json.dumps(b_axis(args.n, M=args.M), indent=1, sort_keys=True))
        return
    res = {"shape": dict(n=args.n, P=args.P, Q=args.Q, b=args.b, M=args.M),
           "model": {name: select_groups_by_model(args.n, args.P, args.Q, args.b, args.M, **pf)
                     for name, pf in PLATFORMS.items()}}
    if not args.no_sample:
        res["sampled"] = select_groups_by_sampling(args.n, args.P, args.Q, args.b, args.M,
                                                   steps=args.steps)
    print(json.dumps(res, indent=1, sort_keys=True))


if __name__ == "__main__":
    main()
