"""Throughput of the batched Generals.io environment step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2|c1|c3] [--obs-layout auto|dense|padded]

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
import re
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402

HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["paper_2606_23348_amd/csrc/kernels.hip", "paper_2606_23348_amd/csrc/features.hip",
                  "paper_2606_23348_amd/csrc/device.hpp", "paper_2606_23348_amd/csrc/internal.hpp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
EXTRAS = ("sustained", "step_alone", "features", "copy", "c1", "c3", "rollout", "served", "pool", "served_mix")


_T0 = time.perf_counter()


def log(msg: str):
    """Progress on stderr (the JSON result is the only stdout line)."""
    print(f"[bench {time.perf_counter() - _T0:7.1f}s] {msg}", file=sys.stderr, flush=True)


def kernel_hash() -> str:
    """First 16 hex digits of the SHA-256 of the kernel sources with their
    comments and white space removed: an edit to either leaves the kernels,
    and so the stored counter readings, as they were."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), encoding="utf-8") as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)     # block comments
        src = re.sub(r"//[^\n]*", " ", src)                    # line comments
        h.update(re.sub(r"\s+", "", src).encode())
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


LDS_BYTES_PER_CLK_CU = 128          # 32 banks x 4 bytes per clock per CU
N_CU, CLK_GHZ = 256, 2.4
LDS_PEAK_GBS = LDS_BYTES_PER_CLK_CU * N_CU * CLK_GHZ     # 78,643 GB/s


def lds_for(wl_name: str, avg_s: float):
    """LDS bandwidth of the step kernel: the LDS's busy cycles on indexed
    operations without the bank-conflict stall cycles (SQ_LDS_IDX_ACTIVE -
    SQ_LDS_BANK_CONFLICT, summed over the CUs, from the committed counter
    summary) x 128 bytes per cycle, per launch, over the kernel's live
    average duration; against 128 B/clk x 256 CUs x 2.4 GHz.  None if the
    counters were taken on another kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f).get(wl_name)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("kernel_hash") != kernel_hash() or "lds_active_cycles" not in rec:
        return None
    busy = rec["lds_active_cycles"] - rec["lds_conflict_cycles"]
    by = busy * LDS_BYTES_PER_CLK_CU
    ach = by / avg_s / 1e9
    return {"achieved": ach, "peak": LDS_PEAK_GBS, "unit": "GB/s", "frac": ach / LDS_PEAK_GBS,
            "bytes_per_launch": by, "bank_conflict_share": rec["lds_conflict_cycles"] / max(1.0, rec["lds_active_cycles"]),
            "source": rec.get("summary")}


def copy_ceiling_gbs(gen, torch, n_bytes: int = 1 << 30, reps: int = 20) -> float:
    """Bandwidth of the library's streaming copy kernel (16-byte nontemporal
    loads and stores; read + write bytes / time): the practical ceiling of
    a read-once / write-once stream next to the 8 TB/s peak."""
    src = torch.empty(n_bytes, dtype=torch.uint8, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    for _ in range(3):
        gen.gen_stream_copy(dst, src, stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        gen.gen_stream_copy(dst, src, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    assert torch.equal(dst[:4096], src[:4096])
    gbs = 2 * n_bytes * reps / (e0.elapsed_time(e1) / 1e3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def spread_ceiling_gbs(gen, torch, ks=(0, 1, 2, 3, 4, 5, 6, 8, 11), n_bytes: int = 8 << 30, reps: int = 20) -> dict:
    """Bandwidth of the library's spread kernel (each 16-byte source chunk
    written to k destination chunks, the copy's form; read + write bytes /
    time) for k writes per read: the practical ceiling of a stream with a
    step's own mix of reads and writes (1v1 24x24 writes about 3.5 times
    what it reads, the mixed pool about 4.4, FFA-8 25x25 about 11).  8 GiB
    written, so that even the k = 11 source (745 MB) is well beyond the
    256 MB Infinity Cache (at 1 GiB the sources of k >= 4 fit in it).
    k = 0: the write-only stream (zeros, nothing read)."""
    dst = torch.empty(n_bytes, dtype=torch.uint8, device="cuda")
    src = torch.empty(n_bytes, dtype=torch.uint8, device="cuda").fill_(1)
    stream = torch.cuda.current_stream()
    out = {}
    for k in ks:
        n_src = -(-(n_bytes // 16) // k) * 16 if k else 0
        for _ in range(3):
            gen.gen_stream_spread(dst, src[:n_src], k, stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            gen.gen_stream_spread(dst, src[:n_src], k, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        out[str(k)] = (n_bytes + n_src) * reps / (e0.elapsed_time(e1) / 1e3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return out


def run_step_alone(b, wl, torch, stream, steps: int, first_step: int) -> dict:
    """gen_step by itself with the actions already in HBM: each step's
    actions come from a separate gen_sample_actions launch that lies
    outside the events timing the step."""
    ev0 = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ev1 = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    for t in range(steps):
        b.sample(wl.actor_seed, first_step + t)
        ev0[t].record(stream)
        b.step()
        ev1[t].record(stream)
    torch.cuda.synchronize()
    ms = np.array([ev0[t].elapsed_time(ev1[t]) for t in range(steps)])
    by = step_bytes(wl)
    alone = by["step"] - 4 * wl.P          # no next-step actions written
    return {"kernel": "k_env<STEP> (gen_step)", "steps": steps, "step_kernel_ms_mean": float(ms.mean()),
            "step_kernel_ms_p50": float(np.percentile(ms, 50)), "step_kernel_ms_p99": float(np.percentile(ms, 99)),
            "frames_per_s": b.n_envs / (float(ms.mean()) / 1e3),
            "achieved_gbs": alone * b.n_envs / (float(ms.mean()) / 1e3) / 1e9, "algorithmic_bytes_per_frame": alone}


def feature_bytes(wl) -> dict:
    """Algorithmic HBM bytes per frame of gen_features: it reads the state,
    the memory header, the per-player memory (1 + 4 + 4 bytes per cell) and
    the 7 earlier frames of the ring (6 bytes per cell each); it writes the
    per-player memory, this frame's ring slot, the header and the float32
    [P][38][H][W] features."""
    HW, P, win = wl.H * wl.W, wl.P, 512
    read = HW * 6 + 32 + 64 + 9 * P * HW + 7 * 6 * HW
    write = 9 * P * HW + 6 * HW + 40 + 38 * 4 * P * HW + 4 + 12 * P
    tok_read = win * 4 + win * 12 * P            # the scoreboard ring, for the 512-turn windows
    tok_write = 2 * win * 4 * P
    return {"read": read, "write": write, "total": read + write,
            "total_with_tokens": read + write + tok_read + tok_write}


def run_features(b, wl, torch, stream, steps: int, first_step: int) -> dict:
    """The 38-channel features (gen_features) after every fused step; only
    the features launch lies between the events."""
    b.features(tokens=True)                       # allocates the memory and the outputs
    ev0 = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ev1 = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    for t in range(steps):
        b.step_sample(wl.actor_seed, first_step + t)
        ev0[t].record(stream)
        b.features(tokens=True)
        ev1[t].record(stream)
    torch.cuda.synchronize()
    ms = np.array([ev0[t].elapsed_time(ev1[t]) for t in range(steps)])
    by = feature_bytes(wl)
    out = {"kernel": "k_features (gen_features, with the temporal tokens)", "steps": steps,
           "kernel_ms_mean": float(ms.mean()), "kernel_ms_p50": float(np.percentile(ms, 50)),
           "frames_per_s": b.n_envs / (float(ms.mean()) / 1e3),
           "algorithmic_bytes_per_frame": by["total_with_tokens"],
           "achieved_gbs": by["total_with_tokens"] * b.n_envs / (float(ms.mean()) / 1e3) / 1e9}
    out["frac_of_peak"] = out["achieved_gbs"] / HBM_PEAK_GBS
    out["traffic"] = traffic_for("features-" + wl.name, b.n_envs)
    b.feat = b.fmem = b.tokens = None
    torch.cuda.empty_cache()
    return out


def run_rollout(gen, torch, n_envs: int = 512, n_steps: int = 512) -> dict:
    """The paper's training setting (512 envs x 512-step rollouts, 1v1 on the
    official 23x23 rules): features, random actor and step per step, into a
    rollout buffer; one timed rollout after a short warm-up."""
    H = W = 23
    params = gen.make_params(0, 2, generator=1, min_general_dist=17, castle_radius=6)
    b = gen.Batch(n_envs, H, W, 0, params, seed=7)
    out = b.rollout(16, 1007, 0, tokens=True)          # warm-up
    del out
    torch.cuda.empty_cache()
    big = {"feat": torch.empty((n_steps, n_envs, 2, 38, H, W), dtype=torch.float32, device="cuda"),
           "tokens": torch.empty((n_steps, n_envs, 2, 2, 512), dtype=torch.float32, device="cuda"),
           "actions": torch.empty((n_steps, n_envs, 2), dtype=torch.int32, device="cuda"),
           "rewards": torch.empty((n_steps, n_envs, 2), dtype=torch.int32, device="cuda"),
           "dones": torch.empty((n_steps, n_envs), dtype=torch.uint8, device="cuda")}
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    b.rollout(n_steps, 1007, 16, tokens=True, out=big)
    e1.record()
    torch.cuda.synchronize()
    s_ = e0.elapsed_time(e1) / 1e3
    del big, b
    torch.cuda.empty_cache()
    return {"workload": f"rollout 1v1 {H}x{W} official rules, {n_envs} envs x {n_steps} steps "
                        "(features + tokens + random actor + step)",
            "ms_per_rollout": s_ * 1e3, "frames_per_s": n_envs * n_steps / s_, "launches": 2 * n_steps + 1}


def pool_rw_per_frame(specs) -> tuple:
    """Mean algorithmic bytes read and written per frame of the pooled step
    (same accounting as step_bytes, per env shape; the scalar record also
    carries the step counter, so 14 live bytes are written)."""
    HW = specs["H"].astype(np.int64) * specs["W"].astype(np.int64)
    P = specs["P"].astype(np.int64)
    read = HW * 6 + 32 + 4 * P + 32          # + the env's 32-byte descriptor
    write = HW * 5 + P * 8 * HW + 4 * P + 1 + 14 + 4 * P
    return float(read.mean()), float(write.mean())


def pool_bytes_per_frame(specs) -> float:
    return sum(pool_rw_per_frame(specs))


_SPREAD = {}          # k writes per read -> GB/s, filled by the copy leg


def practical(achieved_gbs: float, writes_per_read: float):
    """The achieved rate against the practical ceiling of a stream with the
    same ratio of writes to reads (the spread kernel's table, linear between
    its points, the last point beyond them); None without the copy leg."""
    if not _SPREAD:
        return None
    pts = sorted((int(k), v) for k, v in _SPREAD.items() if int(k) >= 1)
    r = writes_per_read
    if r <= pts[0][0]:
        ceil = pts[0][1]
    elif r >= pts[-1][0]:
        ceil = pts[-1][1]
    else:
        for (k0, v0), (k1, v1) in zip(pts, pts[1:]):
            if k0 <= r <= k1:
                ceil = v0 + (v1 - v0) * (r - k0) / (k1 - k0)
                break
    return {"writes_per_read": r, "ceiling_gbs": ceil, "frac": achieved_gbs / ceil,
            "source": "spread_ceiling_gbs (k writes per read, 8 GiB written)"}


def run_pool(gen, torch, steps: int, tune_it: bool) -> dict:
    """The mixed pool in one launch per step, replayed from a captured graph,
    against one plain launch per (H, W, mode) bucket over the same envs."""
    from paper_2606_23348_amd import tune as tuner
    wl = workloads.C4
    specs = workloads.mixed_specs(wl.n_envs, wl.seed)
    common = gen.make_params(0, 2, mountain_thresh=wl.thresh, city_army_min=wl.city_army_min,
                             city_army_max=wl.city_army_max, auto_reset=wl.auto_reset)
    best, table = ({"waves_per_group": 1, "grid": 0, "order": 0}, {})
    if tune_it:
        n_cus = torch.cuda.get_device_properties(0).multi_processor_count
        cands = [{"waves_per_group": w, "grid": gr, "order": o} for o in (0, 1) for w in (1, 2)
                 for gr in (0, 8 * n_cus)]
        best, table = tuner.tune(specs, common, seed=wl.seed, actor_seed=wl.actor_seed, steps=8, cache_path=None,
                                 cands=cands, progress=log)
    buckets, bucket_report = [], {}
    if tune_it:
        buckets, bucket_report = tuner.tune_buckets(specs, common, seed=wl.seed, actor_seed=wl.actor_seed, base=best,
                                                    cache_path=None, progress=log)

    def timed(table) -> float:
        """Seconds per step of graph replays (K steps per graph) with the
        pool-wide packing `best` and the per-bucket table."""
        pool = gen.Pool(specs, common, seed=wl.seed)
        s = torch.cuda.Stream()
        K = 10
        with torch.cuda.stream(s):
            pool.set_tuning(**best, stream=s)
            pool.set_buckets(table, stream=s)
            pool.reset(actor_seed=wl.actor_seed, stream=s)
            pool.capture(K, wl.actor_seed, s)
            pool.replay(s)
            s.synchronize()
            reps = max(1, steps // K)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            for _ in range(reps):
                pool.replay(s)
            e1.record(s)
            s.synchronize()
        del pool
        torch.cuda.empty_cache()
        return e0.elapsed_time(e1) / 1e3 / (reps * K)

    single_s = timed([])
    table_s = timed(buckets) if buckets else single_s
    step_s = min(single_s, table_s)
    rd, wr = pool_rw_per_frame(specs)
    bpf = rd + wr
    achieved = bpf * wl.n_envs / step_s / 1e9
    # baseline: each (H, W, mode, P) bucket as its own plain batch, one launch each per step
    keys = np.stack([specs["H"], specs["W"], specs["mode"], specs["P"]], 1)
    uniq, inv = np.unique(keys, axis=0, return_inverse=True)
    batches = []
    for bi, (H, W, mode, P) in enumerate(uniq):
        n = int((inv == bi).sum())
        first = int(np.flatnonzero(inv == bi)[0])
        prm = gen.make_params(int(mode), int(P), mountain_thresh=wl.thresh, cities_min=int(specs["cities_min"][first]),
                              cities_max=int(specs["cities_max"][first]),
                              min_general_dist=int(specs["min_general_dist"][first]),
                              city_army_min=wl.city_army_min, city_army_max=wl.city_army_max, auto_reset=1)
        b = gen.Batch(n, int(H), int(W), int(mode), prm, seed=wl.seed, env_base=first)
        b.sample(wl.actor_seed, 0)
        batches.append(b)
    log(f"pool: {len(uniq)} per-bucket batches built")
    bsteps = 5
    for b in batches:
        b.step_sample(wl.actor_seed, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(bsteps):
        for b in batches:
            b.step_sample(wl.actor_seed, t + 2)
    torch.cuda.synchronize()
    bucket_s = (time.perf_counter() - t0) / bsteps
    del batches
    torch.cuda.empty_cache()
    return {"workload": wl.name, "n_envs": wl.n_envs, "frames_per_s": wl.n_envs / step_s,
            "ms_per_step": step_s * 1e3, "graph_steps": 10, "tuning": best,
            "tuning_candidates": len(table),
            "per_bucket_tuning": {"table": buckets, "ms_per_step_best_single_packing": single_s * 1e3,
                                  "ms_per_step_per_bucket": table_s * 1e3,
                                  "gain_over_single": single_s / table_s - 1.0, "used": table_s < single_s,
                                  "candidates_us": bucket_report},
            "per_bucket_plain": {"buckets": int(len(uniq)), "frames_per_s": wl.n_envs / bucket_s,
                                 "ms_per_step": bucket_s * 1e3},
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "algorithmic_bytes_per_frame": bpf,
                         "traffic": traffic_for(wl.name, wl.n_envs), "lds": lds_for(wl.name, step_s),
                         "practical": practical(achieved, wr / rd)}}


def served_roofline(frames_per_s: float, specs, key: str | None = None) -> dict:
    """Whole-job served throughput against the HBM peak: frames/s x the
    pooled step's algorithmic bytes per frame of the served envs (a served
    group is a pool: descriptor read and step counter included).  With a
    counter record for `key` taken on the current kernel source, also the
    measured DRAM bytes per frame."""
    rd, wr = pool_rw_per_frame(specs)
    bpf = rd + wr
    ach = frames_per_s * bpf / 1e9
    out = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
           "algorithmic_bytes_per_frame": bpf, "kernel": "k_serve", "traffic_bytes_per_frame": None,
           "practical": practical(ach, wr / rd)}
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f).get(key) if key else None
    except (OSError, ValueError):
        rec = None
    if rec and rec.get("kernel_hash") == kernel_hash():
        out["traffic_bytes_per_frame"] = rec.get("bytes_per_frame")
    return out


def run_served_c2(gen, torch, duration_s: float) -> dict:
    """The headline workload served: its 65,536 envs as 256 groups of 256,
    one closed-loop client per group issuing back-to-back step requests."""
    wl = workloads.C2
    n_clients, per = 256, 256
    specs = {"H": np.full(n_clients * per, wl.H), "W": np.full(n_clients * per, wl.W),
             "mode": np.full(n_clients * per, wl.mode), "P": np.full(n_clients * per, wl.P),
             "cities_min": np.full(n_clients * per, wl.cities_min),
             "cities_max": np.full(n_clients * per, wl.cities_max),
             "min_general_dist": np.full(n_clients * per, wl.min_general_dist)}
    common = gen.make_params(0, 2, **wl.params())
    srv = gen.Server(3 << 30, n_launch_streams=2)
    gaps = np.zeros((n_clients, 1))
    rep = srv.drive(np.full(n_clients, per), specs, seed=wl.seed, actor_seed=wl.actor_seed, gaps_us=gaps,
                    duration_s=duration_s, steps_per_group=0, common=common)
    srv.close_server()
    del srv
    torch.cuda.empty_cache()
    fps = rep["frames"] / rep["wall_s"]
    return {"workload": "served-" + wl.name + " (256 groups x 256 envs, 256 closed-loop clients)",
            "frames_per_s": fps, "requests": rep["requests"],
            "lat_p50_us": rep["lat_p50_us"], "lat_p99_us": rep["lat_p99_us"],
            "envs_per_launch": rep["envs_per_launch"], "launches": rep["launches"], "wall_s": rep["wall_s"],
            "roofline": served_roofline(fps, specs, "served-" + wl.name)}


def run_served_mix(gen, torch, duration_s: float) -> dict:
    """256 clients x 8 groups of 64..2,048 envs with the pooled mix of shapes
    and modes; Poisson arrivals at 4,000 requests/s per client, closed loop
    per group; groups end after 1,000 steps and are replaced."""
    wl = workloads.C5
    n_groups = wl.n_streams * wl.groups_per_stream
    sizes = workloads.group_sizes(wl.seed, n_groups, wl.batch_min, wl.batch_max)
    specs = workloads.mixed_specs(int(sizes.sum()), wl.seed)
    common = gen.make_params(0, 2, mountain_thresh=workloads.mountain_thresh(1, 5), city_army_min=40,
                             city_army_max=50, auto_reset=1)
    gaps = np.stack([workloads.arrival_gaps(wl.arrival_seed, c, 4096, wl.rate_per_stream) * 1e6
                     for c in range(wl.n_streams)])
    arena = 32 << 30
    srv = gen.Server(arena, n_launch_streams=2)
    rep = srv.drive(sizes, specs, seed=wl.seed, actor_seed=wl.actor_seed, gaps_us=gaps, duration_s=duration_s,
                    steps_per_group=wl.steps_per_group, common=common)
    srv.close_server()
    del srv
    torch.cuda.empty_cache()
    return {"workload": wl.name + f" ({wl.n_streams} clients x {wl.groups_per_stream} groups of "
                                  f"{wl.batch_min}-{wl.batch_max} envs, Poisson {wl.rate_per_stream:.0f} req/s each)",
            "resident_envs": int(sizes.sum()), "arena_gb": arena / 2 ** 30,
            "frames_per_s": rep["frames"] / rep["wall_s"], "requests": rep["requests"],
            "lat_p50_us": rep["lat_p50_us"], "lat_p99_us": rep["lat_p99_us"],
            "envs_per_launch": rep["envs_per_launch"], "launches": rep["launches"], "wall_s": rep["wall_s"],
            "roofline": served_roofline(rep["frames"] / rep["wall_s"], specs, "served-" + wl.name)}


LAYOUT_NAMES = {0: "dense [E,P,8,H,W]", 1: "planes padded to 32 bytes (64 above 2 players)"}


def run_plain_leg(gen, torch, wl, steps: int, warmup: int, obs_layout: int = 0) -> dict:
    """Another plain workload in the headline's form: `warmup` untimed
    fused launches, then `steps` timed back to back between one pair of HIP
    events on the launch stream.  obs_layout 1: observation planes padded to
    32 bytes, 64 above 2 players (the algorithmic bytes stay those of the
    dense planes)."""
    b = gen.Batch(wl.n_envs, wl.H, wl.W, wl.mode,
                  gen.make_params(wl.mode, wl.P, obs_layout=obs_layout, **wl.params()), seed=wl.seed)
    stream = torch.cuda.current_stream()
    b.sample(wl.actor_seed, 0)
    for t in range(warmup):
        b.step_sample(wl.actor_seed, t + 1)
    r0, r1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r0.record(stream)
    for t in range(steps):
        b.step_sample(wl.actor_seed, warmup + t + 1)
    r1.record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    avg = r0.elapsed_time(r1) / 1e3 / steps
    by = step_bytes(wl)
    achieved = by["step"] * wl.n_envs / avg / 1e9
    key = wl.name + ("-padded" if obs_layout else "")       # counter records are per layout
    del b
    torch.cuda.empty_cache()
    return {"workload": wl.name, "obs_layout": LAYOUT_NAMES[obs_layout],
            "steps": steps, "warmup": warmup, "frames_per_s": wl.n_envs * steps / elapsed,
            "step_kernel_ms_mean": avg * 1e3,
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "algorithmic_bytes_per_frame": by["step"],
                         "traffic": traffic_for(key, wl.n_envs), "lds": lds_for(key, avg),
                         "practical": practical(achieved, by["step_write"] / by["step_read"])}}


def host_cores() -> int:
    """Host cores this process may use: its CPU affinity, at most 16 (the
    host share of one GPU on the MI355X nodes this runs on)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(wl, n_envs: int, n_steps: int) -> dict:
    """The oracle on the host's cores: one independent shard of n_envs envs
    per thread (env ids of each shard disjoint, as one process per env
    shard would run them; the C oracle releases the GIL), all running the
    whole loop -- random actor, step, observation -- for n_steps steps.  Also
    one shard alone on one thread."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle

    def shard(i, steps):
        cfg = oracle.Config(H=wl.H, W=wl.W, mode=wl.mode, P=wl.P, seed=wl.seed, env_base=i * n_envs, **wl.params())
        st, _ = oracle.reset(cfg, n_envs)
        t0 = time.perf_counter()
        oracle.run(cfg, st, wl.actor_seed, 0, steps)
        return time.perf_counter() - t0

    one = shard(0, n_steps)
    n = host_cores()
    n_steps_each = max(1, n_steps // 4)
    with ThreadPoolExecutor(n) as pool:
        t0 = time.perf_counter()
        list(pool.map(lambda i: shard(i, n_steps_each), range(n)))
        wall = time.perf_counter() - t0
    return {"value": n * n_envs * n_steps_each / wall, "unit": "frames/s", "cores": n, "kind": "oracle",
            "sample": f"{n} threads x {n_envs} envs x {n_steps_each} steps of {wl.name} (random actor + step + "
                      f"observation per frame, each thread its own env shard), {wall:.1f} s wall",
            "one_core": {"value": n_envs * n_steps / one, "unit": "frames/s", "cores": 1,
                         "sample": f"{n_envs} envs x {n_steps} steps on one thread, {one:.1f} s"}}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="c2", choices=sorted(workloads.PLAIN))
    ap.add_argument("--obs-layout", default="auto", choices=["auto", "dense", "padded"],
                    help="observation planes of the timed workload: dense [E,P,8,H,W], or each plane padded "
                         "to 32 bytes (64 above 2 players); auto pads them above 2 players, as pools do")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-envs", type=int, default=1024)
    ap.add_argument("--cpu-steps", type=int, default=400)
    ap.add_argument("--calib-copy", type=int, default=0,
                    help="only run N streaming copies of 1 GiB (counter calibration run) and exit")
    ap.add_argument("--no-extras", action="store_true",
                    help="plain workload only (no served, pooled or copy-ceiling legs)")
    ap.add_argument("--extras", default=",".join(EXTRAS),
                    help="comma-separated subset of the extra legs: " + ",".join(EXTRAS))
    ap.add_argument("--served-seconds", type=float, default=2.0)
    ap.add_argument("--no-tune", action="store_true")
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
            gen.gen_stream_copy(dst, src)          # k_stream_copy: 1 GiB read, 1 GiB written
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes": n, "copies": args.calib_copy}))
        return 0

    wl = workloads.PLAIN[args.workload]
    K = args.steps if args.steps is not None else wl.steps
    W = args.warmup
    E = wl.n_envs
    layout = 1 if args.obs_layout == "padded" or (args.obs_layout == "auto" and wl.P > 2) else 0
    key = wl.name + ("-padded" if layout else "")            # counter records are per layout
    params = gen.make_params(wl.mode, wl.P, obs_layout=layout, **wl.params())
    b = gen.Batch(E, wl.H, wl.W, wl.mode, params, seed=wl.seed)
    stream = torch.cuda.current_stream()

    # actions of step 0; afterwards every launch steps all envs and samples the next actions
    b.sample(wl.actor_seed, 0)
    for t in range(W):
        b.step_sample(wl.actor_seed, t + 1)
    torch.cuda.synchronize()

    # the timed region: K back-to-back launches on one stream, bracketed by a
    # pair of HIP events on that stream (the average launch duration) and by
    # device synchronisation on the host clock (the whole-job throughput)
    r0, r1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r0.record(stream)
    for t in range(K):
        b.step_sample(wl.actor_seed, W + t + 1)
    r1.record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    avg_step_s = r0.elapsed_time(r1) / 1e3 / K

    # per-launch latency, after the timed region: one event pair around each
    # of a few hundred more launches (the events themselves add a little)
    n_lat = min(K, 500)
    ev0 = [torch.cuda.Event(enable_timing=True) for _ in range(n_lat)]
    ev1 = [torch.cuda.Event(enable_timing=True) for _ in range(n_lat)]
    for t in range(n_lat):
        ev0[t].record(stream)
        b.step_sample(wl.actor_seed, W + K + t + 1)
        ev1[t].record(stream)
    torch.cuda.synchronize()
    step_ms = np.array([ev0[t].elapsed_time(ev1[t]) for t in range(n_lat)])
    by = step_bytes(wl)
    achieved = by["step"] * E / avg_step_s / 1e9
    traffic = traffic_for(key, E)
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
                   "obs_layout": LAYOUT_NAMES[layout],
                   "step": "random legal actor + environment step, inputs resident in HBM",
                   "parallelism": "single GPU"},
        "step_kernel_ms": {"mean": avg_step_s * 1e3,
                           "isolated_launch_p50": float(np.percentile(step_ms, 50)),
                           "isolated_launch_p99": float(np.percentile(step_ms, 99)), "isolated_launches": n_lat},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_env<STEP, actor fused> (gen_step_sample)",
                     "algorithmic_bytes_per_frame": by["step"],
                     "frames_per_launch": E, "lds": lds_for(key, avg_step_s)},
    }
    legs = set() if args.no_extras else set(x for x in args.extras.split(",") if x)
    unknown = legs - set(EXTRAS)
    if unknown:
        print(f"unknown extra legs {sorted(unknown)}", file=sys.stderr)
        return 2
    log(f"headline {wl.name}: {value / 1e6:.1f} M frames/s")
    if "sustained" in legs:
        # the same launch, 2,000 more back to back right after the timed
        # region: the rate a long run settles at (the first tens of launches
        # of a fresh process run at a different rate on some boxes)
        n_s = 2000
        q0, q1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        q0.record(stream)
        for t in range(n_s):
            b.step_sample(wl.actor_seed, W + K + n_lat + t + 1)
        q1.record(stream)
        torch.cuda.synchronize()
        s_avg = q0.elapsed_time(q1) / 1e3 / n_s
        out["sustained"] = {"launches": n_s, "step_kernel_ms_mean": s_avg * 1e3, "frames_per_s": E / s_avg,
                            "roofline_frac": by["step"] * E / s_avg / 1e9 / HBM_PEAK_GBS}
    if "step_alone" in legs:
        out["step_alone"] = run_step_alone(b, wl, torch, stream, min(K, 1000), W + K + n_lat + 2001)
    if "features" in legs:
        log("features leg")
        out["features"] = run_features(b, wl, torch, stream, 100, W + K + min(K, 1000) + 1)
    del b
    torch.cuda.empty_cache()
    if "copy" in legs:
        log("copy ceiling")
        out["roofline"]["copy_ceiling_gbs"] = copy_ceiling_gbs(gen, torch)
        _SPREAD.update(spread_ceiling_gbs(gen, torch))
        out["roofline"]["spread_ceiling_gbs"] = dict(_SPREAD)
        out["roofline"]["practical"] = practical(achieved, by["step_write"] / by["step_read"])
        if "sustained" in out:
            out["sustained"]["practical"] = practical(by["step"] * E / (out["sustained"]["step_kernel_ms_mean"] / 1e3)
                                                      / 1e9, by["step_write"] / by["step_read"])
    if "c1" in legs:
        # 16 envs of 10x10: 16 workgroups on 256 CUs, bound by launch latency, not bytes
        out["c1"] = run_plain_leg(gen, torch, workloads.C1, workloads.C1.steps, W)
        out["c1"]["roofline"]["bound"] = "latency (16 workgroups)"
        out["c1"]["roofline"]["practical"] = None
    if "c3" in legs:
        log("FFA-8 leg")
        out["c3"] = run_plain_leg(gen, torch, workloads.C3, max(K, 20), W, obs_layout=1)
        out["c3_dense"] = run_plain_leg(gen, torch, workloads.C3, max(K, 20), W, obs_layout=0)
    if "rollout" in legs:
        log("rollout leg")
        out["rollout"] = run_rollout(gen, torch)
    if "served" in legs:
        log("served leg")
        out["served"] = run_served_c2(gen, torch, args.served_seconds)
    if "pool" in legs:
        log("pool leg")
        out["pool"] = run_pool(gen, torch, 200, not args.no_tune)
    if "served_mix" in legs:
        log("served mix leg")
        out["served_mix"] = run_served_mix(gen, torch, args.served_seconds)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_envs, args.cpu_steps)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
