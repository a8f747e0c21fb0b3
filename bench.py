"""Throughput of the batched Generals.io environment step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2|c1|c3]

One timed step is one pass of the whole hot path over every env of the
workload, one launch of gen_step_sample: the environment step (moves,
combat, captures, growth, terminal, auto-reset, fog, observation, state
store) followed by the random legal actor drawing the next step's actions,
with all inputs resident in HBM.
`value` is frames per second (1 frame = 1 env advanced 1 step).

The JSON line also carries
  roofline      achieved HBM bandwidth of the step kernel (algorithmic bytes /
                its average duration, HIP events on its own stream) against
                the 8 TB/s peak; `traffic` = DRAM bytes per launch measured
                with rocprofv3 counters (profiles/), null if the kernel source
                changed since they were taken.
  cpu_baseline  the CPU oracle (single thread) on a bounded sample of the
                same workload, in frames per second.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402

HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["paper_2606_23348_amd/csrc/kernels.hip", "paper_2606_23348_amd/csrc/device.hpp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def step_bytes(wl) -> dict:
    """Algorithmic HBM bytes per frame of the step kernel and of the actor.

    The fused step reads the env's state (owner int8, type uint8, army int32
    per cell, the 32-byte scalar record) and its P actions; it writes owner
    and army, the uint8 [P][8][H][W] observation, P rewards, the done byte,
    the 10 live bytes of the scalar record and the P actions of the next step
    (type is written only after a capture or a reset).
    """
    HW, P = wl.H * wl.W, wl.P
    read = HW * (1 + 1 + 4) + 32 + 4 * P
    write = HW * (1 + 4) + P * 8 * HW + 4 * P + 1 + 10 + 4 * P      # + the next step's actions
    return {"step_read": read, "step_write": write, "step": read + write}


def traffic_for(wl_name: str, n_launch_frames: int):
    """DRAM bytes per step launch from the committed counter summary, if it
    was taken on the current kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    rec = t.get(wl_name)
    if not rec or rec.get("kernel_hash") != kernel_hash():
        return None
    return rec.get("bytes_per_launch")


def copy_ceiling_gbs(torch, n_bytes: int = 1 << 30, reps: int = 10) -> float:
    """Bandwidth of a plain device-to-device copy (read + write bytes / time):
    the practical streaming ceiling next to the 8 TB/s peak."""
    src = torch.empty(n_bytes, dtype=torch.uint8, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * n_bytes * reps / (e0.elapsed_time(e1) / 1e3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def cpu_baseline(wl, n_envs: int, n_steps: int) -> dict:
    import oracle
    cfg = oracle.Config(H=wl.H, W=wl.W, mode=wl.mode, P=wl.P, seed=wl.seed, **wl.params())
    st, _ = oracle.reset(cfg, n_envs)
    t0 = time.perf_counter()
    oracle.run(cfg, st, wl.actor_seed, 0, n_steps)
    dt = time.perf_counter() - t0
    return {"value": n_envs * n_steps / dt, "unit": "frames/s", "cores": 1, "kind": "oracle",
            "sample": f"{n_envs} envs x {n_steps} steps of {wl.name} (sample + step + observe per frame), "
                      f"{dt:.1f} s on one host thread"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="c2", choices=sorted(workloads.PLAIN))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-envs", type=int, default=1024)
    ap.add_argument("--cpu-steps", type=int, default=400)
    ap.add_argument("--calib-copy", type=int, default=0,
                    help="only run N copies of 1 GiB (counter calibration run) and exit")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the environment step has no cross-GPU work, and this "
              "build runs on a single MI355X (use --gpus 1)", file=sys.stderr)
        return 2

    import torch
    import paper_2606_23348_amd as gen

    torch.cuda.set_device(0)
    if args.calib_copy:
        n = 1 << 30
        src = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        for _ in range(args.calib_copy):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes": n, "copies": args.calib_copy}))
        return 0

    wl = workloads.PLAIN[args.workload]
    K = args.steps if args.steps is not None else wl.steps
    W = args.warmup
    E = wl.n_envs
    params = gen.make_params(wl.mode, wl.P, **wl.params())
    b = gen.Batch(E, wl.H, wl.W, wl.mode, params, seed=wl.seed)
    stream = torch.cuda.current_stream()

    # actions of step 0; afterwards every launch steps all envs and samples the next actions
    b.sample(wl.actor_seed, 0)
    for t in range(W):
        b.step_sample(wl.actor_seed, t + 1)
    torch.cuda.synchronize()

    ev0 = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    ev1 = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(K):
        ev0[t].record(stream)
        b.step_sample(wl.actor_seed, W + t + 1)
        ev1[t].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    step_ms = np.array([ev0[t].elapsed_time(ev1[t]) for t in range(K)])
    avg_step_s = float(step_ms.mean()) / 1e3
    by = step_bytes(wl)
    achieved = by["step"] * E / avg_step_s / 1e9
    traffic = traffic_for(wl.name, E)
    value = E * K / elapsed

    out = {
        "metric": "frames/s (1v1 24x24, 64K envs) plain vs served; p50/p99 step latency",
        "value": value,
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": elapsed / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": wl.name, "n_envs": E, "H": wl.H, "W": wl.W,
                   "mode": {0: "1v1", 1: "2v2", 2: "ffa"}[wl.mode], "players": wl.P,
                   "step": "random legal actor + environment step, inputs resident in HBM",
                   "parallelism": "single GPU"},
        "step_kernel_ms": {"mean": float(step_ms.mean()), "p50": float(np.percentile(step_ms, 50)),
                           "p99": float(np.percentile(step_ms, 99))},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_env<STEP, actor fused> (gen_step_sample)",
                     "algorithmic_bytes_per_frame": by["step"],
                     "frames_per_launch": E, "copy_ceiling_gbs": copy_ceiling_gbs(torch)},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_envs, args.cpu_steps)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
