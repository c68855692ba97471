#!/usr/bin/env python
"""Benchmark: Newton-CG body-steps/sec, forward step + adjoint, on the batched-strips workload.

One bench step = one full backprop-through-time pass over the batch: 512 strips of uneven size
(4s x s quads, s ~ U{4..32}, 128 to 8192 triangles), 50 backward-Euler steps forward
(isb_step, Newton-PCG to 1e-6 relative residual), then 50 adjoint solves (isb_solve_adjoint,
CG to 1e-6, each starting from the adjoint of the step after) and parameter VJPs (isb_vjp_params)
backward, loss = -sum of the bodies' centre of mass x. value = bodies x steps / seconds for the batched mixed-precision persistent solver.
Beside it: the plain single-body FP64 GPU path on a 64-body subset (8 bodies per size octile), the
FP64 CPU oracle on a bounded sample of the same bodies (one single-threaded process per host core),
the error of every leg against the oracle's stored results (tests/golden/, written by scripts that
call only oracle/), and the roofline of the dominant kernel (the persistent step launch), timed
with HIP events on the stream the library launches on, beside its measured HBM traffic.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

# the oracle leg is timed single-threaded
for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ.setdefault(_v, "1")

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
HERE = os.path.dirname(os.path.abspath(__file__))
TRAFFIC_PROFILE = os.path.join(HERE, "profiles", "batched_strips_512_hbm_counters.md")
TRAFFIC_PROFILE_4096 = os.path.join(HERE, "profiles", "batched_strips_4096_hbm_counters.md")
GOLDEN = os.path.join(HERE, "tests", "golden", "bench_reference.json")
TET_GOLDEN = os.path.join(HERE, "tests", "golden", "tet_block_step.json")
MAX_POOL = 16  # host cores of one GPU's share of the machine
METRIC = "Newton-CG steps/sec fwd+adjoint, batched FP32/64 vs plain FP64, 1e-6 residual"


# the sources the batched persistent kernel is compiled from (its body logic, the element and
# spring math, the device helpers and data layout, the ABI header)
BATCHED_SOURCES = ("isb_batched.hip", "isb_batched_kernel.hpp", "isb_batched_k2.hip", "isb_batched_k3.hip",
                   "isb_body.hpp", "isb_device.hpp", "isb_elem.hpp", "isb_spring.hpp", "isb_internal.hpp", "isb.h")


def kernel_source_hash(files=BATCHED_SOURCES):
    """sha256 over the named library sources (name and contents, in the order given): a
    measured-traffic figure in profiles/ applies only while this matches the hash recorded with it."""
    import hashlib
    h = hashlib.sha256()
    src = os.path.join(HERE, "paper_2102_05791_amd", "csrc")
    for name in files:
        path = os.path.join(HERE, "include", name) if name == "isb.h" else os.path.join(src, name)
        h.update(name.encode() + b"\0")
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel_mode, profile=None):
    """HBM bytes per launch of the batched kernel (mode 0 step, 1 adjoint) from the committed
    FETCH_SIZE / WRITE_SIZE summary (the 512-body one unless `profile` names another), or None when
    the sources changed since it was taken."""
    try:
        with open(profile or TRAFFIC_PROFILE) as fh:
            rec = next(json.loads(l.split("traffic-record:", 1)[1]) for l in fh if "traffic-record:" in l)
    except (OSError, StopIteration, ValueError):
        return None
    if rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch", {}).get(str(kernel_mode))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed bench steps (full BPTT passes)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--bodies", type=int, default=512)
    ap.add_argument("--rollout", type=int, default=50, help="time steps per BPTT pass")
    ap.add_argument("--plain-bodies", type=int, default=64, help="octile subset for the plain FP64 path")
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--cpu-bodies", type=int, default=64, help="octile subset for the CPU oracle leg")
    ap.add_argument("--cpu-steps", type=int, default=10)
    ap.add_argument("--mall-bodies", type=int, default=4096,
                    help="bodies of the leg whose working set exceeds the 256 MB last-level cache (0: skip)")
    ap.add_argument("--mall-rollout", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--block", type=int, default=0, help="batched workgroup size (0 = library default)")
    ap.add_argument("--profile", action="store_true", help="one untimed pass only (for rocprofv3)")
    ap.add_argument("--profile-elements", action="store_true",
                    help="the element kernels alone on the --elem-grid mesh in wave order (for rocprofv3)")
    ap.add_argument("--profile-tet", action="store_true",
                    help="the tet block's CG, resident and with two launches per iteration, 1 + 2 steps "
                         "fwd + adjoint each, with every CG iteration counted (for rocprofv3)")
    ap.add_argument("--no-tet", action="store_true", help="skip the 3D tet-block leg")
    ap.add_argument("--no-graph", action="store_true", help="skip the graph-replay leg")
    ap.add_argument("--no-policy", action="store_true", help="skip the policy-training leg")
    ap.add_argument("--no-springs", action="store_true", help="skip the vertex-pair spring leg")
    ap.add_argument("--no-energies", action="store_true", help="skip the alternative-energy legs")
    ap.add_argument("--no-first-order", action="store_true", help="skip the Newton vs first-order leg")
    ap.add_argument("--first-order-steps", type=int, default=5)
    ap.add_argument("--policy-iters", type=int, default=4)
    ap.add_argument("--tet-steps", type=int, default=20)
    ap.add_argument("--no-elem-roofline", action="store_true", help="skip the size-R element roofline leg")
    ap.add_argument("--elem-grid", type=str, default="192x128x64", help="Kuhn-tet grid of the size-R leg")
    return ap.parse_args()


# ---------------------------------------------------------------------------------------------
# algorithmic bytes (minimal traffic: every array element moved once per pass)
# ---------------------------------------------------------------------------------------------
def elem_bytes(dim, word, compact=False):
    """conn + rest data + actuation, per element: the general record holds Dm^-1, the fibre vector
    and W mu, W lam, W k_f; the compact one (uniform material, fibre along an axis) Dm^-1 and W."""
    rest = dim * dim + 1 if compact else dim * dim + dim + 3
    return 4 * (dim + 1) + word * (rest + 1)


def hv_state_bytes(dim, word):
    """Per-element state the Hessian-vector pass reads at a Newton iterate: the symmetric 4x4
    Hessian with respect to the edge matrix for triangles (10 words), F and F d for tetrahedra."""
    return word * (10 if dim == 2 else dim * dim + dim)


def hv_elem_bytes(dim, word, compact=False):
    """Element bytes of one batched Hessian-vector pass: 16-bit body-local connectivity + the
    stored state (triangles), or + rest data + actuation + the stored F, F d (tetrahedra)."""
    if dim == 2:
        return 2 * (dim + 1) + hv_state_bytes(dim, word)
    return elem_bytes(dim, word, compact) - 2 * (dim + 1) + hv_state_bytes(dim, word)


def cg_iter_bytes(dim, ne, nv, word_hv, compact=False):
    """One batched CG iteration: the Hessian-vector element pass (p is in LDS), and the x/r update
    pass (xs, r read and written, the FP32 preconditioner and the vertex diagonal in the element
    precision read); the direction pass touches LDS only."""
    return hv_elem_bytes(dim, word_hv, compact) * ne + (32 + 4 + word_hv) * nv * dim


def trial_bytes(dim, ne, nv, word_hv, compact=False):
    """One fused line-search trial: 16-bit connectivity, FP64 rest data and actuation, E(x) read,
    E(x_t) written, the Hessian-vector state stored per element; x, dx, x0, xhat, pinned read and G
    (FP64), the vertex diagonal (element precision) and the FP32 preconditioner written per DOF;
    mass and c_v per vertex."""
    return ((elem_bytes(dim, 8, compact) - 2 * (dim + 1) + 16 + hv_state_bytes(dim, word_hv)) * ne
            + (41 + 8 + 4 + word_hv) * nv * dim + 16 * nv)


def spring_hv_bytes(dim, word):
    """One spring in a batched Hessian-vector pass: two 16-bit ends and the stored block K."""
    return 4 + word * dim * (dim + 1) // 2


def spring_trial_bytes(dim, word):
    """One spring in a trial (or diagonal) pass: ends, stiffness, 1/l0 and action (FP64), its energy
    read and written, the block K stored."""
    return 4 + 24 + 16 + word * dim * (dim + 1) // 2


def step_launch_bytes(dim, ne, nv, st, word_hv, ns=0, compact=False):
    """Algorithmic bytes of one body (ne elements, nv vertices, ns springs) in one step launch,
    from its solver statistics."""
    dof = nv * dim
    trials = 1 + st["newton_iters"] + st["ls_backtracks"]
    setup = 57 * dof + 16 * nv                 # x0, v0, pinned -> xhat, x; c_v; v1 at the end
    per_newton = (8 + 4 + word_hv + 24) * dof + 16 * dof + 24 * dof  # CG start; g.dx; x += alpha dx
    return (setup + trials * (trial_bytes(dim, ne, nv, word_hv, compact) + ns * spring_trial_bytes(dim, word_hv))
            - 8 * (ne + ns) + st["newton_iters"] * per_newton
            + st["cg_iters"] * (cg_iter_bytes(dim, ne, nv, word_hv, compact) + ns * spring_hv_bytes(dim, word_hv)))


def adjoint_launch_bytes(dim, ne, nv, st, word_hv, ns=0, warm=False, compact=False):
    """Right-hand side (xbar, vbar, pinned -> G; c_v), the FP64 diagonal pass that also stores the
    Hessian-vector state, the warm start (one Hessian-vector pass over the given w; w read, G read
    and written, the vertex diagonal read, w parked and added back), the CG start and the CG
    iterations."""
    dof = nv * dim
    rhs = 25 * dof + 16 * nv
    diag = ((elem_bytes(dim, 8, compact) - 2 * (dim + 1) + hv_state_bytes(dim, word_hv)) * ne + (9 + 4 + word_hv) * dof
            + 16 * nv + ns * (spring_trial_bytes(dim, word_hv) - 16))
    start = (hv_elem_bytes(dim, word_hv, compact) * ne + ns * spring_hv_bytes(dim, word_hv)
             + (8 + 16 + word_hv + 8 + 24) * dof) if warm else 0
    return (rhs + diag + start + (36 + 4 + word_hv) * dof
            + st["adj_cg_iters"] * (cg_iter_bytes(dim, ne, nv, word_hv, compact) + ns * spring_hv_bytes(dim, word_hv)))


def octile_pick(sizes, n):
    """n bodies, n/8 per octile of the size distribution, evenly spaced in size order within each."""
    order = np.argsort(np.asarray(sizes), kind="stable")
    per = max(1, n // 8)
    pick = []
    for q in np.array_split(order, 8):
        if len(q):
            pick.extend(q[np.linspace(0, len(q) - 1, min(per, len(q))).round().astype(int)].tolist())
    return np.asarray(pick, dtype=np.int64)


def golden():
    with open(GOLDEN) as fh:
        return json.load(fh)


def sampled_error(x, ref, x0=None):
    """Relative error of the state x (full array) against a stored oracle sample: over the sampled
    vertices, relative to the full displacement norm stored with it (or the sampled values)."""
    vs = np.asarray(ref["vertices"])
    key = "x1" if "x1" in ref else "x"
    gx = np.asarray(ref[key])
    d = np.linalg.norm(x[vs] - gx)
    if x0 is not None:
        return float(d / np.linalg.norm(gx - x0[vs]))
    return float(d / np.linalg.norm(gx))


# ---- the CPU oracle leg: one single-threaded process per host core ---------------------------
_CPU_W = None


def _oracle_body(job):
    """One body of the batched workload through the FP64 oracle (a worker of the CPU leg): the
    forward steps (Newton with direct solves, to the benchmark's tolerance) and the backward pass
    (direct adjoint of Eq. 9 and the VJPs) of L = -COM_x."""
    from oracle import solve as osolve
    from oracle.fem import Problem
    b, steps = job
    wb = _CPU_W.body(int(b))
    wb.scene.update(tol_rel=_CPU_W.scene["tol_rel"])
    p = Problem.from_workload(wb)
    t = time.perf_counter()
    states, _ = osolve.rollout(p, wb.x0, wb.v0, wb.actions[:steps], tol=wb.scene["tol_rel"])
    osolve.rollout_grad(p, states, wb.actions[:steps], osolve.com_x_loss_grad(p, states[-1][0]))
    return int(b), int(wb.n_e), steps, time.perf_counter() - t


def start_cpu_pool(w):
    """Fork the oracle's worker processes before the GPU is used (they never touch it)."""
    import multiprocessing as mp
    global _CPU_W
    _CPU_W = w
    n = max(1, min(os.cpu_count() or 1, MAX_POOL))
    return mp.get_context("fork").Pool(n), n


def cpu_leg(pool, n_proc, w, args):
    nb = w.n_bodies
    cpick = octile_pick(np.diff(w.body_e_off), min(args.cpu_bodies, nb))
    tc = time.perf_counter()
    done = 0
    for b, ne, steps, dt in pool.imap_unordered(_oracle_body, [(int(b), args.cpu_steps) for b in cpick]):
        done += steps
    tcpu = time.perf_counter() - tc
    pool.close()
    pool.join()
    print(f"# oracle leg done: {len(cpick)} bodies x {args.cpu_steps} steps in {tcpu:.1f} s on {n_proc} processes",
          file=sys.stderr, flush=True)
    return {"value": round(done / tcpu, 3), "unit": "body-steps/s", "cores": n_proc, "kind": "oracle",
            "sample": f"{len(cpick)} bodies (8 per size octile) x {args.cpu_steps} steps of the batched "
                      f"workload, forward Newton (SuperLU) to {w.scene['tol_rel']} + adjoint + VJP, one "
                      f"single-threaded process per core, {tcpu:.1f} s wall",
            "host_cpus": os.cpu_count()}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: there is no multi-GPU path (asked for --gpus {args.gpus}). "
              "Bodies are independent, so a multi-GPU run would give each process (one per GPU) a "
              "slice of the bodies balanced by elements and iterations, with no exchange during a "
              "solve.", file=sys.stderr)
        sys.exit(2)
    from synth import scenes
    from synth.meshes import concat_bodies
    T = args.rollout
    w = scenes.batched_strips(args.bodies, steps=T)
    pool = None
    if not (args.no_cpu or args.profile or args.profile_elements or args.profile_tet):
        pool, n_proc = start_cpu_pool(w)
    import torch
    from paper_2102_05791_amd import Context, isb

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.profile_tet:
        print(json.dumps({"profile_pass": "tet_block", **tet_profile_pass(torch, Context, isb, scenes)}))
        return
    if args.profile_elements:
        out = element_roofline_mesh(args.elem_grid, torch, Context, isb, scenes, block_order=False)
        src = torch.ones(2 ** 27, dtype=torch.float64, device=dev)   # byte-counter calibration copy
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"profile_pass": "elements", "copy_bytes_each_way": 2 ** 30, **out}))
        return
    nb = w.n_bodies
    ctx = Context.from_workload(w, precision="mixed", solver=1)
    if args.block:
        ctx.set_option(isb.OPT_BLOCK, args.block)
    ctx.set_option(isb.OPT_GRAPH_SAFE, 1)
    x0 = torch.tensor(w.x0, dtype=torch.float64, device=dev)
    v0 = torch.tensor(w.v0, dtype=torch.float64, device=dev)
    acts = torch.tensor(w.actions, dtype=torch.float64, device=dev)
    mass = ctx.mass()
    body_of_v = torch.tensor(np.repeat(np.arange(nb), np.diff(w.body_v_off)), device=dev)
    msum = torch.zeros(nb, dtype=torch.float64, device=dev).index_add_(0, body_of_v, mass)
    xbar_T = torch.zeros_like(x0)
    xbar_T[:, 0] = -mass / msum[body_of_v]      # L = -sum_b COM_x(body b)

    step_ev, adj_ev = [], []

    def bptt(record=False, stats=False):
        xs, vs = [x0], [v0]
        st_f, st_a = [], []
        for t in range(T):
            if record:
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
            x1, v1, s, _ = ctx.step(xs[-1], vs[-1], acts[t], stats=stats)
            if record:
                e1.record()
                step_ev.append((e0, e1))
            xs.append(x1)
            vs.append(v1)
            st_f.append(s)
        xb, vb = xbar_T, torch.zeros_like(x0)
        a_bar = torch.empty_like(acts)
        wv = None  # each adjoint CG starts from the adjoint of the step after, in place
        for t in range(T - 1, -1, -1):
            if record:
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
            wv, s, _ = ctx.solve_adjoint(xs[t + 1], xs[t], acts[t], xb, vb, stats=stats, w=wv, w_init=wv)
            if record:
                e1.record()
                adj_ev.append((e0, e1))
            out = ctx.vjp_params(wv, xs[t + 1], xs[t], acts[t], vb, want=("a_bar", "x0_bar", "v0_bar"))
            a_bar[t] = out["a_bar"]
            xb, vb = out["x0_bar"], out["v0_bar"]
            st_a.append(s)
        return xs, a_bar, st_f, st_a

    if args.profile:
        bptt()
        # calibration for hardware byte counters: a plain 1 GiB device-to-device copy
        src = torch.ones(2 ** 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"profile_pass": "done", "bodies": nb, "rollout": T, "copy_bytes_each_way": 2 ** 30}))
        return

    for _ in range(args.warmup):
        bptt()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pass_ev = []
    for k in range(args.steps):
        p0, p1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        p0.record()
        xs, a_bar, _, _ = bptt(record=True)
        p1.record()
        pass_ev.append((p0, p1))
        print(f"# timed step {k + 1}/{args.steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_median = float(np.median([a.elapsed_time(b) for a, b in pass_ev]))
    ms_per_step = 1e3 * wall / args.steps
    body_steps = nb * T * args.steps
    value = body_steps / wall
    step_ms = float(np.mean([a.elapsed_time(b) for a, b in step_ev]))
    adj_ms = float(np.mean([a.elapsed_time(b) for a, b in adj_ev]))

    # solver statistics of one pass (untimed: statistics force a host read per launch)
    _, _, st_f, st_a = bptt(stats=True)
    print("# statistics pass done", file=sys.stderr, flush=True)
    ne_b, nv_b = np.diff(w.body_e_off), np.diff(w.body_v_off)
    cr = ctx.get_option(isb.INFO_COMPACT_AXIS) >= 0
    fb = [sum(step_launch_bytes(2, ne_b[b], nv_b[b], s[b], 4, compact=cr) for b in range(nb)) for s in st_f]
    # st_a runs backward in time: the first adjoint starts from zero, every later one from the last w
    ab = [sum(adjoint_launch_bytes(2, ne_b[b], nv_b[b], s[b], 4, warm=k > 0, compact=cr) for b in range(nb))
          for k, s in enumerate(st_a)]
    it = {"newton_per_step": float(np.mean([[s["newton_iters"] for s in S] for S in st_f])),
          "cg_per_step": float(np.mean([[s["cg_iters"] for s in S] for S in st_f])),
          "adj_cg_per_step": float(np.mean([[s["adj_cg_iters"] for s in S] for S in st_a])),
          "max_newton": int(np.max([[s["newton_iters"] for s in S] for S in st_f])),
          "not_converged_steps": int(sum(1 for S in st_f for s in S if not (s["flags"] & 1))),
          "stagnated_steps": int(sum(1 for S in st_f for s in S if s["flags"] & 2)),
          "fp64_fallback_steps": int(sum(1 for S in st_f for s in S if s["flags"] & 16)),
          "adj_not_converged": int(sum(1 for S in st_a for s in S if not (s["flags"] & 8)))}
    dominant = "step" if step_ms >= adj_ms else "adjoint"
    roofline = batched_roofline(fb, ab, step_ms, adj_ms, None)

    # error against the oracle's stored first step of sampled bodies (tol 1e-13); the bench solves
    # to the metric's 1e-6 relative residual
    parity = None
    if nb == 512:
        x1 = xs[1].cpu().numpy()
        errs = []
        for ref in golden()["batched_strips_512"]:
            b = ref["body"]
            sv = slice(w.body_v_off[b], w.body_v_off[b + 1])
            errs.append(sampled_error(x1[sv], ref, w.x0[sv]))
        parity = {"bodies": [r["body"] for r in golden()["batched_strips_512"]],
                  "x1_rel_err_vs_oracle_displacement": errs,
                  "note": "batched mixed first step at tol 1e-6 vs the oracle's at 1e-13 (tests/golden/"
                          "bench_reference.json), over 128 sampled vertices per body"}

    # plain single-body FP64 GPU path on an octile subset (same bodies, one at a time)
    plain = None
    if not args.no_plain and args.plain_bodies > 0:
        pick = octile_pick(ne_b, min(args.plain_bodies, nb))
        parts = [(w.body(int(b)).X, w.body(int(b)).T, w.body(int(b)).pinned) for b in pick]
        X, Tm, P, vo, eo = concat_bodies(parts)
        sub = scenes.Workload("plain_subset", 2, X, Tm, P, np.concatenate([w.body(int(b)).mu for b in pick]),
                              np.concatenate([w.body(int(b)).lam for b in pick]),
                              np.concatenate([w.body(int(b)).kf for b in pick]),
                              np.concatenate([w.body(int(b)).fdir for b in pick]),
                              np.concatenate([w.body(int(b)).rho for b in pick]), dict(w.scene), X.copy(),
                              np.zeros_like(X), np.concatenate([w.body(int(b)).actions for b in pick], axis=1),
                              vo, eo)
        pctx = Context.from_workload(sub, precision="fp64", solver=0)
        px0 = torch.tensor(sub.x0, dtype=torch.float64, device=dev)
        pv0 = torch.zeros_like(px0)
        pa = torch.tensor(sub.actions, dtype=torch.float64, device=dev)
        pm = pctx.mass()

        def plain_pass(S):
            xs_, vs_ = [px0], [pv0]
            for t in range(S):
                x1_, v1_, _, _ = pctx.step(xs_[-1], vs_[-1], pa[t], stats=False)
                xs_.append(x1_)
                vs_.append(v1_)
            xb_, vb_ = torch.zeros_like(px0), torch.zeros_like(px0)
            xb_[:, 0] = -pm / pm.sum()
            wv_ = None
            for t in range(S - 1, -1, -1):
                wv_, _, _ = pctx.solve_adjoint(xs_[t + 1], xs_[t], pa[t], xb_, vb_, stats=False, w=wv_, w_init=wv_)
                out_ = pctx.vjp_params(wv_, xs_[t + 1], xs_[t], pa[t], vb_, want=("a_bar", "x0_bar", "v0_bar"))
                xb_, vb_ = out_["x0_bar"], out_["v0_bar"]

        plain_pass(1)
        torch.cuda.synchronize()
        print("# plain FP64 warm-up pass done", file=sys.stderr, flush=True)
        tp = time.perf_counter()
        plain_pass(args.plain_steps)
        torch.cuda.synchronize()
        tpl = time.perf_counter() - tp
        pv = len(pick) * args.plain_steps / tpl
        plain = {"value": round(pv, 2), "unit": "body-steps/s", "bodies": int(len(pick)),
                 "steps": args.plain_steps, "sample": "8 bodies per size octile (evenly spaced in size order)",
                 "dtype": "f64", "solver": "plain host-driven Newton-PCG, grid-wide kernels",
                 "batched_over_plain": round(value / pv, 1)}

    ceiling = copy_ceiling(torch, isb)
    roofline["copy_ceiling"] = ceiling
    roofline["frac_of_copy_ceiling"] = round(roofline["achieved"] / ceiling["GBs"], 4)
    print("# copy ceiling done", file=sys.stderr, flush=True)
    # the same BPTT pass captured once as a HIP graph (graph-safe mode, no statistics) and replayed
    graph = None
    if not args.no_graph:
        g = torch.cuda.CUDAGraph()
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            gxs, ga_bar, _, _ = bptt()
        g.replay()
        torch.cuda.synchronize()
        tg = time.perf_counter()
        for _ in range(args.steps):
            g.replay()
        torch.cuda.synchronize()
        tgw = time.perf_counter() - tg
        gdiff = float((ga_bar - a_bar).abs().max() / a_bar.abs().max())
        graph = {"value": round(nb * T * args.steps / tgw, 1), "unit": "body-steps/s",
                 "ms_per_step": round(1e3 * tgw / args.steps, 3), "replays": args.steps,
                 "a_bar_max_rel_diff_vs_eager": gdiff,
                 "note": "whole BPTT pass (50 step launches, 50 adjoint launches, VJPs) captured once and replayed"}
        del g
        print("# graph replay leg done", file=sys.stderr, flush=True)

    springs = None if args.no_springs else spring_leg(args, torch, Context, isb, scenes)
    energies = None if args.no_energies else energy_leg(args, torch, Context, isb, scenes)
    first_order = None if args.no_first_order else first_order_leg(args, torch, Context, isb, scenes)
    policy = None if args.no_policy else policy_leg(args, torch, Context, isb, scenes)
    tet = None if args.no_tet else tet_leg(args, torch, Context, isb, scenes)
    elem = None if args.no_elem_roofline else element_roofline_leg(args, torch, Context, isb, scenes)
    mall = None if args.mall_bodies <= 0 else mall_leg(args, torch, Context, isb, scenes, ceiling)
    # the FP64 CPU oracle last, on the processes forked before the GPU was used (idle until now)
    cpu = None if pool is None else cpu_leg(pool, n_proc, w, args)
    if elem:
        for part in (elem, elem["tet_block_64x32x32"]):
            for prec in ("fp64", "mixed", "gradient_fp64"):
                part[prec]["frac_of_copy_ceiling"] = round(part[prec]["achieved_GBs"] / ceiling["GBs"], 4)

    line = {"metric": METRIC, "value": round(value, 1), "unit": "body-steps/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
            "ms_per_step_median": round(ms_median, 3),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
            "data": "synthetic",
            "config": {"workload": f"batched_strips: {nb} bodies (4s x s quads, s~U{{4..32}}, "
                                   f"{w.n_e} triangles, {w.n_v} vertices), {T} backward-Euler steps "
                                   "fwd + adjoint + VJP per bench step",
                       "solver": "batched persistent, mixed FP32 element Hv / FP64 vectors",
                       "tol_rel": w.scene["tol_rel"], "adj_tol_rel": w.scene["adj_tol_rel"],
                       "block": ctx.get_option(isb.OPT_BLOCK)},
            "iterations": it, "plain_fp64": plain, "parity": parity, "roofline": roofline,
            "cpu_baseline": cpu, "graph_replay": graph, "springs": springs, "energies": energies,
            "first_order": first_order, "policy_training": policy, "tet_block": tet, "element_roofline": elem,
            "beyond_last_level_cache": mall}
    print(json.dumps(line))


def batched_roofline(fb, ab, step_ms, adj_ms, profile):
    """Roofline of the batched solver's dominant launch: the design's algorithmic bytes (every array
    the launch must move, once per pass; the CG direction and accumulator stay in LDS) over the
    HIP-event launch time, beside the measured traffic (calibrated FETCH_SIZE + WRITE_SIZE from the
    committed counter summary) over the same time."""
    dominant = "step" if step_ms >= adj_ms else "adjoint"
    mode = 0 if dominant == "step" else 1
    dom_ms = step_ms if mode == 0 else adj_ms
    dom_bytes = float(np.mean(fb if mode == 0 else ab))
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9
    traffic = measured_traffic(mode, profile)
    t_adj = measured_traffic(1, profile)
    meas = None if traffic is None else traffic / (dom_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "achieved_measured": None if meas is None else round(meas, 1),
            "frac_measured": None if meas is None else round(meas / HBM_PEAK_GBS, 4),
            "kernel": f"k_batched<2,float,{mode}> ({dominant} launch)",
            "launch_ms": round(dom_ms, 4), "algorithmic_bytes_per_launch": int(dom_bytes),
            "step_launch_ms": round(step_ms, 4), "adjoint_launch_ms": round(adj_ms, 4),
            "adjoint_launch": {"algorithmic_bytes_per_launch": int(np.mean(ab)),
                               "achieved": round(float(np.mean(ab)) / (adj_ms * 1e-3) / 1e9, 1),
                               "frac": round(float(np.mean(ab)) / (adj_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                               "traffic": t_adj,
                               "frac_measured": None if t_adj is None
                               else round(t_adj / (adj_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}}


def mall_leg(args, torch, Context, isb, scenes, ceiling):
    """The batched workload at 4096 bodies (8x the headline's): one CG iteration's working set is
    about 8x 136 MB, beyond the 256 MB last-level cache, so the step launch streams from HBM. A
    BPTT pass of --mall-rollout steps (forward + adjoint + VJPs), timed per launch."""
    dev = torch.device("cuda:0")
    T = args.mall_rollout
    w = scenes.batched_strips(args.mall_bodies, steps=T)
    nb = w.n_bodies
    ctx = Context.from_workload(w, precision="mixed", solver=1)
    ctx.set_option(isb.OPT_GRAPH_SAFE, 1)
    x0 = torch.tensor(w.x0, dtype=torch.float64, device=dev)
    v0 = torch.zeros_like(x0)
    acts = torch.tensor(w.actions, dtype=torch.float64, device=dev)
    mass = ctx.mass()
    body_of_v = torch.tensor(np.repeat(np.arange(nb), np.diff(w.body_v_off)), device=dev)
    msum = torch.zeros(nb, dtype=torch.float64, device=dev).index_add_(0, body_of_v, mass)
    xbar_T = torch.zeros_like(x0)
    xbar_T[:, 0] = -mass / msum[body_of_v]
    step_ev, adj_ev = [], []

    def bptt(record=False, stats=False):
        xs, vs, st_f, st_a = [x0], [v0], [], []
        for t in range(T):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            x1, v1, sf, _ = ctx.step(xs[-1], vs[-1], acts[t], stats=stats)
            e1.record()
            if record:
                step_ev.append((e0, e1))
            xs.append(x1)
            vs.append(v1)
            st_f.append(sf)
        xb, vb, wv = xbar_T, torch.zeros_like(x0), None
        for t in range(T - 1, -1, -1):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            wv, sa, _ = ctx.solve_adjoint(xs[t + 1], xs[t], acts[t], xb, vb, stats=stats, w=wv, w_init=wv)
            e1.record()
            if record:
                adj_ev.append((e0, e1))
            out = ctx.vjp_params(wv, xs[t + 1], xs[t], acts[t], vb, want=("a_bar", "x0_bar", "v0_bar"))
            xb, vb = out["x0_bar"], out["v0_bar"]
            st_a.append(sa)
        return st_f, st_a

    bptt()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bptt(record=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = float(np.mean([a.elapsed_time(b) for a, b in step_ev]))
    adj_ms = float(np.mean([a.elapsed_time(b) for a, b in adj_ev]))
    st_f, st_a = bptt(stats=True)
    ne_b, nv_b = np.diff(w.body_e_off), np.diff(w.body_v_off)
    cr = ctx.get_option(isb.INFO_COMPACT_AXIS) >= 0
    fb = [sum(step_launch_bytes(2, ne_b[b], nv_b[b], S[b], 4, compact=cr) for b in range(nb)) for S in st_f]
    ab = [sum(adjoint_launch_bytes(2, ne_b[b], nv_b[b], S[b], 4, warm=k > 0, compact=cr) for b in range(nb))
          for k, S in enumerate(st_a)]
    roof = batched_roofline(fb, ab, step_ms, adj_ms, TRAFFIC_PROFILE_4096)
    roof["frac_of_copy_ceiling"] = round(roof["achieved"] / ceiling["GBs"], 4)
    print("# beyond-cache leg done", file=sys.stderr, flush=True)
    return {"workload": f"batched_strips: {nb} bodies ({w.n_e} triangles, {w.n_v} vertices), {T} backward-Euler "
                        "steps fwd + adjoint + VJP, batched mixed, graph-safe",
            "value": round(nb * T / wall, 1), "unit": "body-steps/s", "ms_per_pass": round(1e3 * wall, 3),
            "newton_per_step": float(np.mean([[s["newton_iters"] for s in S] for S in st_f])),
            "cg_per_step": float(np.mean([[s["cg_iters"] for s in S] for S in st_f])),
            "adj_cg_per_step": float(np.mean([[s["adj_cg_iters"] for s in S] for S in st_a])),
            "not_converged_steps": int(sum(1 for S in st_f for s in S if not (s["flags"] & 1))),
            "roofline": roof}


def copy_ceiling(torch, isb):
    """HBM ceiling measured with the library's streaming copy kernel: 2 GiB copied, median of 10."""
    n = 1 << 28
    src = torch.ones(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        isb.stream_copy(src, dst)
    torch.cuda.synchronize()
    ts = []
    for _ in range(10):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        isb.stream_copy(src, dst)
        e1.record()
        ts.append((e0, e1))
    torch.cuda.synchronize()
    ms = float(np.median([a.elapsed_time(b) for a, b in ts]))
    gbs = 2 * 8 * n / (ms * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return {"kernel": "isb_stream_copy", "bytes_moved": 2 * 8 * n, "ms": round(ms, 4), "GBs": round(gbs, 1),
            "frac_of_8TBs": round(gbs / HBM_PEAK_GBS, 4)}


def spring_leg(args, torch, Context, isb, scenes):
    """The batched workload with the fibres as vertex-pair springs (passive triangles, one spring per
    horizontal grid edge): the same BPTT pass (T steps fwd + T adjoints + VJPs), batched mixed."""
    dev = torch.device("cuda:0")
    T = args.rollout
    w = scenes.batched_spring_strips(args.bodies, steps=T)
    nb = w.n_bodies
    ctx = Context.from_workload(w, precision="mixed", solver=1)
    ctx.set_option(isb.OPT_GRAPH_SAFE, 1)
    x0 = torch.tensor(w.x0, dtype=torch.float64, device=dev)
    v0 = torch.zeros_like(x0)
    acts = torch.tensor(w.actions, dtype=torch.float64, device=dev)
    mass = ctx.mass()
    body_of_v = torch.tensor(np.repeat(np.arange(nb), np.diff(w.body_v_off)), device=dev)
    msum = torch.zeros(nb, dtype=torch.float64, device=dev).index_add_(0, body_of_v, mass)
    xbar_T = torch.zeros_like(x0)
    xbar_T[:, 0] = -mass / msum[body_of_v]
    step_ev = []

    def bptt(record=False, stats=False):
        xs, vs, st_f, st_a = [x0], [v0], [], []
        for t in range(T):
            if record:
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
            x1, v1, sf, _ = ctx.step(xs[-1], vs[-1], acts[t], stats=stats)
            if record:
                e1.record()
                step_ev.append((e0, e1))
            xs.append(x1)
            vs.append(v1)
            st_f.append(sf)
        xb, vb = xbar_T, torch.zeros_like(x0)
        wv = None
        for t in range(T - 1, -1, -1):
            wv, sa, _ = ctx.solve_adjoint(xs[t + 1], xs[t], acts[t], xb, vb, stats=stats, w=wv, w_init=wv)
            out = ctx.vjp_params(wv, xs[t + 1], xs[t], acts[t], vb, want=("a_bar", "x0_bar", "v0_bar"))
            xb, vb = out["x0_bar"], out["v0_bar"]
            st_a.append(sa)
        return xs, st_f, st_a

    bptt()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        xs, _, _ = bptt(record=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = float(np.mean([a.elapsed_time(b) for a, b in step_ev]))
    _, st_f, st_a = bptt(stats=True)
    ne_b, nv_b, ns_b = np.diff(w.body_e_off), np.diff(w.body_v_off), np.diff(w.body_s_off)
    cr = ctx.get_option(isb.INFO_COMPACT_AXIS) >= 0
    fb = float(np.mean([sum(step_launch_bytes(2, ne_b[b], nv_b[b], S[b], 4, ns_b[b], compact=cr) for b in range(nb))
                        for S in st_f]))
    achieved = fb / (step_ms * 1e-3) / 1e9
    errs, bodies = [], []
    if nb == 512:
        x1 = xs[1].cpu().numpy()
        for ref in golden()["batched_spring_strips_512"]:
            b = ref["body"]
            sv = slice(w.body_v_off[b], w.body_v_off[b + 1])
            errs.append(sampled_error(x1[sv], ref, w.x0[sv]))
            bodies.append(b)
    print("# spring leg done", file=sys.stderr, flush=True)
    return {"workload": f"batched_spring_strips: {nb} bodies, {w.n_e} passive triangles + {w.n_s} springs, "
                        f"{w.n_v} vertices, {T} backward-Euler steps fwd + adjoint + VJP",
            "value": round(nb * T * args.steps / wall, 1), "unit": "body-steps/s",
            "ms_per_step": round(1e3 * wall / args.steps, 3), "solver": "batched mixed, graph-safe",
            "step_launch_ms": round(step_ms, 4),
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(achieved / HBM_PEAK_GBS, 4), "algorithmic_bytes_per_launch": int(fb)},
            "newton_per_step": float(np.mean([[s["newton_iters"] for s in S] for S in st_f])),
            "cg_per_step": float(np.mean([[s["cg_iters"] for s in S] for S in st_f])),
            "adj_cg_per_step": float(np.mean([[s["adj_cg_iters"] for s in S] for S in st_a])),
            "not_converged_steps": int(sum(1 for S in st_f for s in S if not (s["flags"] & 1))),
            "x1_rel_err_vs_oracle_displacement": {"bodies": bodies, "err": errs,
                                                  "note": "first step at tol 1e-6 vs the oracle's at 1e-13"}}


def energy_leg(args, torch, Context, isb, scenes):
    """The batched workload with each alternative isotropic energy (Sec. 3): one warm-up and one
    timed BPTT pass (T steps fwd + T adjoints + VJPs), batched mixed; error of body 0's first step
    against the oracle."""
    dev = torch.device("cuda:0")
    T = args.rollout
    out = {}
    for model in ("stvk", "corot", "snh"):
        w = scenes.batched_strips(args.bodies, steps=T)
        w.model = model
        nb = w.n_bodies
        ctx = Context.from_workload(w, precision="mixed", solver=1)
        ctx.set_option(isb.OPT_GRAPH_SAFE, 1)
        x0 = torch.tensor(w.x0, dtype=torch.float64, device=dev)
        v0 = torch.zeros_like(x0)
        acts = torch.tensor(w.actions, dtype=torch.float64, device=dev)
        xbar_T = torch.zeros_like(x0)
        xbar_T[:, 0] = -1.0 / w.n_v
        ev = []

        def bptt(record=False, stats=False):
            xs, vs, sts = [x0], [v0], []
            for t in range(T):
                if record:
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record()
                x1, v1, sf, _ = ctx.step(xs[-1], vs[-1], acts[t], stats=stats)
                if record:
                    e1.record()
                    ev.append((e0, e1))
                xs.append(x1)
                vs.append(v1)
                sts.append(sf)
            xb, vb = xbar_T, torch.zeros_like(x0)
            wv = None
            for t in range(T - 1, -1, -1):
                wv, _, _ = ctx.solve_adjoint(xs[t + 1], xs[t], acts[t], xb, vb, stats=False, w=wv, w_init=wv)
                o = ctx.vjp_params(wv, xs[t + 1], xs[t], acts[t], vb, want=("a_bar", "x0_bar", "v0_bar"))
                xb, vb = o["x0_bar"], o["v0_bar"]
            return xs, sts

        bptt()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xs, _ = bptt(record=True)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        _, sts = bptt(stats=True)
        err = None
        if nb == 512:
            sv = slice(w.body_v_off[0], w.body_v_off[1])
            err = sampled_error(xs[1].cpu().numpy()[sv], golden()["energies"][model], w.x0[sv])
        out[model] = {"value": round(nb * T / wall, 1), "unit": "body-steps/s",
                      "step_launch_ms": round(float(np.mean([a.elapsed_time(b) for a, b in ev])), 4),
                      "newton_per_step": float(np.mean([[s["newton_iters"] for s in S] for S in sts])),
                      "cg_per_step": float(np.mean([[s["cg_iters"] for s in S] for S in sts])),
                      "not_converged_steps": int(sum(1 for S in sts for s in S if not (s["flags"] & 1))),
                      "x1_rel_err_vs_oracle_body0": err}
        del ctx
        print(f"# energy leg {model} done", file=sys.stderr, flush=True)
    out["workload"] = (f"batched_strips: {args.bodies} bodies, {T} backward-Euler steps fwd + adjoint + VJP, "
                       "batched mixed, one timed pass per model")
    return out


def first_order_leg(args, torch, Context, isb, scenes):
    """Newton-PCG against the first-order forward solver (L-BFGS with the same line search and stop,
    the paper's kind of forward pass) on the 64x16 strip, plain FP64 path, at the same relative
    residual: steps/s, iterations and gradient evaluations per step, and the gap between the two
    trajectories."""
    dev = torch.device("cuda:0")
    S = args.first_order_steps
    w = scenes.be_strip(64, 16, steps=S)
    out = {"workload": f"be_strip 64x16 ({w.n_e} triangles), {S} backward-Euler steps, plain FP64, "
                       f"tol_rel {w.scene['tol_rel']}"}
    finals = {}
    for name, fwd in (("newton_pcg", isb.FORWARD_NEWTON), ("lbfgs", isb.FORWARD_LBFGS)):
        ctx = Context.from_workload(w, precision="fp64", solver=0)
        ctx.set_option(isb.OPT_FORWARD, fwd)
        acts = torch.tensor(w.actions, dtype=torch.float64, device=dev)
        x = torch.tensor(w.x0, dtype=torch.float64, device=dev)
        v = torch.zeros_like(x)
        ctx.step(x, v, acts[0], stats=False)    # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its, cgs, lss = [], [], []
        for t in range(S):
            x, v, st, _ = ctx.step(x, v, acts[t])
            its.append(st[0]["newton_iters"])
            cgs.append(st[0]["cg_iters"])
            lss.append(st[0]["ls_backtracks"])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        finals[name] = x.cpu().numpy()
        # gradient evaluations: one per accepted iterate plus the initial one; Newton adds one
        # Hessian-vector product per CG iteration
        out[name] = {"steps_per_s": round(S / dt, 3), "ms_per_step": round(1e3 * dt / S, 2),
                     "iterations_per_step": float(np.mean(its)), "cg_per_step": float(np.mean(cgs)),
                     "backtracks_per_step": float(np.mean(lss))}
        del ctx
    d = finals["lbfgs"] - finals["newton_pcg"]
    out["x_rel_diff_after_steps"] = float(np.linalg.norm(d) / np.linalg.norm(finals["newton_pcg"] - w.x0))
    ref = golden()["be_strip_64x16_5_steps"]
    if ref["steps"] == S:
        for name in ("newton_pcg", "lbfgs"):
            out[name]["x_rel_err_vs_oracle_displacement"] = sampled_error(finals[name], ref, w.x0)
        out["oracle_note"] = f"state after {S} steps at tol 1e-6 vs the oracle's at 1e-13, 128 sampled vertices"
    out["newton_speedup"] = round(out["newton_pcg"]["steps_per_s"] / out["lbfgs"]["steps_per_s"], 1)
    print("# first-order leg done", file=sys.stderr, flush=True)
    return out


def policy_leg(args, torch, Context, isb, scenes):
    """Policy-in-the-loop training (one Adam step per 100-step episode) on the 64x16 strip with the
    batched mixed solver: training iterations per second and the rewards."""
    from paper_2102_05791_amd.policy import FibrePolicy, train_locomotion
    w = scenes.be_strip(64, 16, steps=1)
    dev = torch.device("cuda:0")
    ctx = Context.from_workload(w, precision="mixed", solver=1)
    ctx.set_option(isb.OPT_GRAPH_SAFE, 1)
    x0 = torch.tensor(w.x0, dtype=torch.float64, device=dev)
    v0 = torch.zeros_like(x0)
    H = 100
    # the seeded policy's first episode and its gradient, against the oracle's (stored)
    from paper_2102_05791_amd.policy import episode_reward
    pol = FibrePolicy(ctx.mass(), 2, w.n_e, seed=0)
    r = episode_reward(ctx, pol, x0, v0, H)
    r.backward()
    g = np.concatenate([t.grad.detach().cpu().numpy().ravel() for t in pol.parameters()])
    ref = golden()["policy_strip_64x16"]
    probe = np.random.default_rng([210205791, 7, 1000]).standard_normal(g.size)
    err = {"reward_rel_err": abs(float(r.detach()) - ref["reward"]) / abs(ref["reward"]),
           "grad_norm_rel_err": abs(float(np.linalg.norm(g)) - ref["grad_norm"]) / ref["grad_norm"],
           "grad_probe_rel_err": abs(float(g @ probe) - ref["grad_dot_probe"]) / abs(ref["grad_dot_probe"]),
           "note": "first episode of the seeded policy, batched mixed at tol 1e-6 vs the oracle at 1e-13"}
    pol = FibrePolicy(ctx.mass(), 2, w.n_e, seed=0)
    train_locomotion(ctx, pol, x0, v0, horizon=H, iterations=1)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rewards = train_locomotion(ctx, pol, x0, v0, horizon=H, iterations=args.policy_iters)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print("# policy leg done", file=sys.stderr, flush=True)
    return {"workload": f"be_strip 64x16 ({w.n_e} triangles), episode of {H} backward-Euler steps",
            "policy": "32 ReLU units, FP64; Adam lr 1e-3, one step per episode",
            "iterations_per_s": round(args.policy_iters / dt, 3), "iterations": args.policy_iters,
            "rewards": [round(r, 6) for r in rewards], "solver": "batched mixed, graph-safe",
            "error_vs_oracle": err}


def tet_leg(args, torch, Context, isb, scenes):
    """3D tet block (393,216 tets): plain grid-wide path, mixed, T steps forward + T adjoints."""
    dev = torch.device("cuda:0")
    w = scenes.tet_block(steps=args.tet_steps)
    w = w.permute_elements(isb.wave_order(3, w.n_v, w.T, w.body_e_off))
    ctx = Context.from_workload(w, precision="mixed", solver=0)
    x0 = torch.tensor(w.x0, device=dev)
    v0 = torch.tensor(w.v0, device=dev)
    acts = torch.tensor(w.actions, device=dev)
    m = ctx.mass()

    def run(S, stats, c=None):
        c = c or ctx
        xs, vs, st = [x0], [v0], []
        for t in range(S):
            x1, v1, s, _ = c.step(xs[-1], vs[-1], acts[t], stats=stats)
            xs.append(x1)
            vs.append(v1)
            st.append(s)
        xb = torch.zeros_like(x0)
        xb[:, 0] = -m / m.sum()
        vb = torch.zeros_like(x0)
        sa = []
        wv = None
        for t in range(S - 1, -1, -1):
            wv, s, _ = c.solve_adjoint(xs[t + 1], xs[t], acts[t], xb, vb, stats=stats, w=wv, w_init=wv)
            out = c.vjp_params(wv, xs[t + 1], xs[t], acts[t], vb, want=("a_bar", "x0_bar", "v0_bar"))
            xb, vb = out["x0_bar"], out["v0_bar"]
            sa.append(s)
        return st, sa

    # error of the first step against the oracle's (stored at sampled vertices, tol 1e-12)
    with open(TET_GOLDEN) as fh:
        g = json.load(fh)
    x1, v1, _, _ = ctx.step(x0, v0, acts[0], stats=False)
    x1 = x1.cpu().numpy()
    vs = np.asarray(g["vertices"])
    tet_err = {"x1_rel_err_vs_oracle_displacement": float(np.linalg.norm(x1[vs] - np.asarray(g["x1"])) /
                                                          np.linalg.norm(np.asarray(g["x1"]) - w.x0[vs])),
               "v1_rel_err": float(np.linalg.norm(v1.cpu().numpy()[vs] - np.asarray(g["v1"])) /
                                   np.linalg.norm(np.asarray(g["v1"]))),
               "note": "first step at tol 1e-6 vs the oracle's at 1e-12 (tests/golden/tet_block_step.json)"}
    resident = ctx.get_option(isb.INFO_RESIDENT) > 0 and ctx.get_option(isb.OPT_CG_RESIDENT) == 1

    def warm(c=None):
        # untimed steps for at least 0.1 s, so that the timed steps run at the core clock of a long
        # simulation (the clock rises over tens of milliseconds of sustained load)
        t = time.perf_counter()
        while True:
            run(1, False, c)
            torch.cuda.synchronize()
            if time.perf_counter() - t >= 0.1:
                break

    warm()
    t0 = time.perf_counter()
    run(args.tet_steps, False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st, sa = run(2, True)
    # the same steps with the single-reduction CG as two launches per iteration (the resident solve off)
    launched = None
    if resident:
        ctx.set_option(isb.OPT_CG_RESIDENT, 0)
        warm()
        t1 = time.perf_counter()
        run(args.tet_steps, False)
        torch.cuda.synchronize()
        launched = round(args.tet_steps / (time.perf_counter() - t1), 3)
        ctx.set_option(isb.OPT_CG_RESIDENT, 1)
    # the same steps in FP64 (every product in FP64; resident CG where the body's plan fits)
    ctx64 = Context.from_workload(w, precision="fp64", solver=0)
    warm(ctx64)
    t2 = time.perf_counter()
    run(args.tet_steps, False, ctx64)
    torch.cuda.synchronize()
    fp64_rate = round(args.tet_steps / (time.perf_counter() - t2), 3)
    fp64_resident = ctx64.get_option(isb.INFO_RESIDENT) > 0 and ctx64.get_option(isb.OPT_CG_RESIDENT) == 1
    del ctx64
    print("# tet-block leg done", file=sys.stderr, flush=True)
    cg_its = float(np.mean([s[0]["cg_iters"] for s in st])) + float(np.mean([s[0]["adj_cg_iters"] for s in sa]))
    # one mixed CG iteration by the per-unit bytes of the measurement plan: Hessian-vector product
    # (element word 4 B: conn + Dm^-1 + W + a, 60 B per tet; x, p in and Hp out, 36 B per vertex) and
    # 13 FP64 words of CG vectors per DOF
    it_bytes = w.n_e * (4 * 4 + 4 * (9 + 2)) + w.n_v * 3 * 3 * 4 + 13 * 8 * 3 * w.n_v
    it_us = dt / args.tet_steps / cg_its * 1e6
    cg_form = ("single-reduction, resident (one cooperative launch per solve)" if resident else
               "single-reduction, two launches per iteration" if ctx.get_option(isb.OPT_CG_SINGLE_REDUCTION)
               else "classic")
    return {"workload": f"tet_block 64x32x32 Kuhn tets ({w.n_e} tets, {w.n_v} vertices; block order, then "
                        f"isb_wave_order), {args.tet_steps} backward-Euler steps fwd + adjoint + VJP",
            "solver": "plain grid-wide Newton-PCG, mixed", "value": round(args.tet_steps / dt, 3),
            "unit": "steps/s", "seconds": round(dt, 3),
            "newton_per_step": float(np.mean([s[0]["newton_iters"] for s in st])),
            "cg_per_step": float(np.mean([s[0]["cg_iters"] for s in st])),
            "adj_cg_per_step": float(np.mean([s[0]["adj_cg_iters"] for s in sa])),
            "cg_form": cg_form, "launch_per_iteration_steps_per_s": launched,
            "fp64": {"value": fp64_rate, "unit": "steps/s",
                     "cg_form": "resident" if fp64_resident else "launch per iteration"},
            "cg_iteration": {"us_upper_bound": round(it_us, 2),
                             "note": "whole step time (Newton passes, line search, VJP included) over the "
                                     "forward and adjoint CG iterations",
                             "bytes_per_iteration": it_bytes,
                             "frac_of_8TBs_at_that_rate": round(it_bytes / (it_us * 1e-6) / 8e12, 4)},
            "error_vs_oracle": tet_err}


def tet_profile_pass(torch, Context, isb, scenes):
    """For a kernel trace of the tet block's CG: 2 backward-Euler steps forward + 2 adjoints with the
    resident single-reduction CG, then the same with two launches per iteration, each after one
    untimed warm-up step; reports every CG iteration each form ran, so that a trace's kernel time
    divides into time per iteration."""
    dev = torch.device("cuda:0")
    w = scenes.tet_block(steps=2)
    w = w.permute_elements(isb.wave_order(3, w.n_v, w.T, w.body_e_off))
    ctx = Context.from_workload(w, precision="mixed", solver=0)
    x0 = torch.tensor(w.x0, device=dev)
    v0 = torch.tensor(w.v0, device=dev)
    acts = torch.tensor(w.actions, device=dev)
    m = ctx.mass()
    out = {"workload": f"tet_block ({w.n_e} tets, {w.n_v} vertices), mixed"}
    for form, resident in (("resident", 1), ("two_launches", 0)):
        ctx.set_option(isb.OPT_CG_RESIDENT, resident)
        its, solves = 0, 0
        for steps in (1, 2):
            xs, vs = [x0], [v0]
            for t in range(steps):
                x1, v1, s, _ = ctx.step(xs[-1], vs[-1], acts[t], stats=True)
                xs.append(x1)
                vs.append(v1)
                its += s[0]["cg_iters"]
                solves += s[0]["newton_iters"]
            xb = torch.zeros_like(x0)
            xb[:, 0] = -m / m.sum()
            vb = torch.zeros_like(x0)
            wv = None
            for t in range(steps - 1, -1, -1):
                wv, s, _ = ctx.solve_adjoint(xs[t + 1], xs[t], acts[t], xb, vb, stats=True, w=wv, w_init=wv)
                its += s[0]["adj_cg_iters"]
                solves += 1
                o = ctx.vjp_params(wv, xs[t + 1], xs[t], acts[t], vb, want=("a_bar", "x0_bar", "v0_bar"))
                xb, vb = o["x0_bar"], o["v0_bar"]
        torch.cuda.synchronize()
        out[form] = {"cg_iterations": int(its), "cg_solves_at_least": int(solves),
                     "resident_bodies": int(ctx.get_option(isb.INFO_RESIDENT)) if resident else 0}
    return out


def element_roofline_leg(args, torch, Context, isb, scenes):
    """Element Hessian-vector kernel alone (isb_hessvec_elements, FP64 and mixed) and the element
    gradient kernel alone (isb_gradient_elements, FP64) on a mesh whose element data exceeds the
    256 MB last-level cache; algorithmic bytes / HIP-event time."""
    out = element_roofline_mesh(args.elem_grid, torch, Context, isb, scenes)
    # the same kernels on the 64x32x32 tet block (whose element data fits the last-level cache)
    out["tet_block_64x32x32"] = element_roofline_mesh("64x32x32", torch, Context, isb, scenes)
    print("# element roofline leg done", file=sys.stderr, flush=True)
    return out


def element_roofline_mesh(grid, torch, Context, isb, scenes, block_order=True):
    """The element kernels on one Kuhn-tet grid, with the elements in the order isb_wave_order gives
    the 4x4x4-cube block order (the figures reported), and in the block order itself."""
    from synth import meshes
    dev = torch.device("cuda:0")
    nx, ny, nz = (int(v) for v in grid.split("x"))
    X, Tm = meshes.tet_grid(nx, ny, nz)
    n_e, n_v = Tm.shape[0], X.shape[0]
    rng = np.random.default_rng([210205791, 6])
    x = torch.tensor(X + 0.01 * rng.standard_normal(X.shape), device=dev)
    p = torch.tensor(rng.standard_normal(X.shape), device=dev)
    a_np = meshes.contraction_actuation(rng, n_e)
    perm = isb.wave_order(3, n_v, Tm)
    out = {"mesh": f"tet_grid {nx}x{ny}x{nz}: {n_e} tets, {n_v} vertices; 4x4x4-cube block element order, "
                   "then isb_wave_order inside each patch",
           "timing": f"per kernel: untimed launches for at least {ELEM_WARMUP_S} s and {ELEM_WARMUP_MIN_LAUNCHES} "
                     f"launches, then the median of {ELEM_TIMED_LAUNCHES} launches (HIP events)"}
    out.update(element_times(X, np.ascontiguousarray(Tm[perm]), x, p, torch.tensor(a_np[perm], device=dev),
                             torch, Context, scenes))
    if block_order:
        blk = element_times(X, Tm, x, p, torch.tensor(a_np, device=dev), torch, Context, scenes)
        out["block_order"] = {k: {"launch_ms": v["launch_ms"], "frac_of_8TBs": v["frac_of_8TBs"]}
                              for k, v in blk.items()}
    return out


ELEM_WARMUP_S = 0.1            # element kernels: untimed launches for at least this long ...
ELEM_WARMUP_MIN_LAUNCHES = 20  # ... and at least this many, before the 20 timed ones
ELEM_TIMED_LAUNCHES = 20


def element_times(X, Tm, x, p, a, torch, Context, scenes):
    from synth import meshes
    n_e, n_v = Tm.shape[0], X.shape[0]
    mu, lam = scenes.lame(1e5, 0.45)

    def median_ms(fn):
        # a sustained warm-up, as inside a CG solve that runs the product hundreds of times in a row:
        # the core clock rises under load over tens of milliseconds, and the LDS-bound products follow
        # it (after 3 launches the FP64 product at 9.4 M tets takes 0.25 ms, after 200 0.215 ms; the
        # HBM-bound gradient does not change). The 20 launches after it are the timed ones.
        t0, n = time.perf_counter(), 0
        while n < ELEM_WARMUP_MIN_LAUNCHES or time.perf_counter() - t0 < ELEM_WARMUP_S:
            fn()
            n += 1
            if n % 20 == 0:
                torch.cuda.synchronize()
        torch.cuda.synchronize()
        evs = []
        for _ in range(ELEM_TIMED_LAUNCHES):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            evs.append((e0, e1))
        torch.cuda.synchronize()
        return float(np.median([e0.elapsed_time(e1) for e0, e1 in evs]))

    def rec(ms, byt, kbyt, per_elem, per_vert):
        gbs = byt / (ms * 1e-3) / 1e9
        return {"launch_ms": round(ms, 4), "algorithmic_bytes": int(byt), "achieved_GBs": round(gbs, 1),
                "frac_of_8TBs": round(gbs / HBM_PEAK_GBS, 4), "element_bytes": per_elem, "vertex_bytes": per_vert,
                "kernel_bytes": int(kbyt), "kernel_frac_of_8TBs": round(kbyt / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}

    out = {}
    for prec, word in (("fp64", 8), ("mixed", 4)):
        ctx = Context(0, prec)
        ctx.mesh_upload(3, X, Tm, None)
        ctx.material_upload(np.full(n_e, mu), np.full(n_e, lam), np.full(n_e, 1e5), meshes.x_fibres(n_e, 3),
                            np.ones(n_e), scenes.scene("be", h=1.0 / 30.0))
        compact = ctx.get_option(isb_mod().INFO_COMPACT_AXIS) >= 0
        hp = torch.zeros_like(x)
        ms = median_ms(lambda: ctx.hessvec_elements(x, a, p, hp))
        # algorithmic bytes per Hessian-vector product (the workload's minimal traffic): connectivity,
        # Dm^-1, W and the actuation per element in the element word; x, p in and Hp out per vertex
        eb, vb = 4 * 4 + word * (9 + 2), 3 * 3 * word
        # what this kernel moves at least: 16-bit patch connectivity, Dm^-1 and W in the element word
        # (the compact record), the FP64 actuation; x and p (FP64) in, Hp (FP64) read and written
        keb = 8 + word * (10 if compact else 16) + 8
        out[prec] = rec(ms, n_e * eb + n_v * vb, n_e * keb + n_v * 3 * 32, eb, vb)
        if prec == "fp64":
            # the element gradient (FP64 in both precisions): element data once, x in, g out
            g = torch.zeros_like(x)
            gms = median_ms(lambda: ctx.gradient_elements(x, a, g))
            out["gradient_fp64"] = rec(gms, n_e * (16 + 8 * 11) + n_v * 48, n_e * keb + n_v * 3 * 24, 16 + 88, 48)
        out[prec]["compact_rest_record"] = compact
        del ctx
        torch.cuda.empty_cache()
    return out


def isb_mod():
    from paper_2102_05791_amd import isb
    return isb


if __name__ == "__main__":
    main()
