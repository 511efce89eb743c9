"""Benchmark: EDT + exact local thickness + per-object measures on one MI355X.

Workload (default): a 512^3 uint16 label volume with ~2000 superellipsoids
(semi-axes U[4,30], exponents U[0.3,1], value-noise surface perturbation), the
synthetic stand-in for the paper's labelled micro-CT volume.  A step is one pass of
the whole path over the resident volume (lt_pipeline: EDT, local thickness with
the per-object sums fused into its paint pass, closed forms).  Prints one JSON
line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "voxels/s + objects/s for EDT+local thickness+measures at 512³; % HBM peak"

# Peak of plain 32-bit vector ALU work: 256 CUs x 4 SIMDs x 16 lanes per clock
# (one wave64 VALU instruction per CU per clock) at 2.4 GHz.
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12


# Algorithmic bytes per launch of the streaming kernels for uint16 labels: each
# kernel's inputs read once and outputs written once (neighbour re-reads served by
# caches excluded).  n = voxels, f = fraction of object voxels.
def kernel_bytes(name: str, n: int, f: float, label_bytes: int = 2) -> float | None:
    lb = label_bytes
    table = {
        "edt_pass_x": (lb + 2) * n,                 # labels -> g (uint16)
        "edt_pass_y": (2 + lb + 4) * n,             # g, labels -> d2
        "edt_pass_z": (4 + lb + 4) * n,             # d2, labels -> D
        "bbox_runs": lb * n,                        # labels
        "prune3d": 4 * n + lb * f * n + 4 * n + 4 * (1 - f) * n,   # D, object labels -> kept field; LT = 0 outside
        "fronts3d": 4 * n + 16 * f * n,             # kept field -> 4 front planes of object voxels
        "paint_tiles": (lb + 16 + 4 + 4) * f * n,   # labels, fronts, D (shell test) of object voxels -> LT
        "object_sums": (lb + 4) * n,                # labels + LT
    }
    return table.get(name)


def lattice_tables(dmax: int):
    """N[d] = #{q in Z^3 : |q|^2 < d} and, for the neighbour offsets o with |o|^2 =
    1, 2, 3, T_c[d] = max{|q - o|^2 : |q|^2 < d} (-1 for d = 0), d = 0..dmax."""
    R = int(np.ceil(np.sqrt(dmax))) + 1
    r = np.arange(-R, R + 1)
    qz, qy, qx = np.meshgrid(r, r, r, indexing="ij")
    q2 = (qx * qx + qy * qy + qz * qz).ravel()
    order = np.argsort(q2, kind="stable")
    q2s = q2[order]
    d = np.arange(dmax + 1)
    N = np.searchsorted(q2s, d, side="left")             # points with |q|^2 < d
    T = []
    for o in ((1, 0, 0), (1, 1, 0), (1, 1, 1)):
        e = ((qx - o[0]) ** 2 + (qy - o[1]) ** 2 + (qz - o[2]) ** 2).ravel()[order]
        pm = np.maximum.accumulate(e)
        T.append(np.where(N > 0, pm[np.maximum(N - 1, 0)], -1))
    return N.astype(np.int64), np.stack(T).astype(np.int64)


def ball_cover_work(lab, D) -> tuple[int, int]:
    """Ball-cover algorithmic work of the 3D local thickness: the sum over kept
    centres x of |B(x)| = #{q : |q - x|^2 < D(x)}; a centre is dropped when its open
    ball lies inside the open ball of a 26-neighbour of the same label
    (T_|o|^2[D(x)] < D(y)).  Computed with torch tensor ops on the resident fields
    (outside any timed region).  Returns (work, kept centres)."""
    import torch
    dmax = int(D.max())
    N, T = lattice_tables(dmax)
    Nt = torch.from_numpy(N).to(D.device)
    Tt = torch.from_numpy(T).to(D.device)
    Dl = D.long()
    L = lab.int()
    obj = L != 0
    covered = torch.zeros_like(obj)
    Z, Y, X = D.shape
    Tc = [Tt[c][Dl] for c in range(3)]
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                c = abs(dz) + abs(dy) + abs(dx)
                if c == 0:
                    continue
                def sl(a, o, n):
                    return slice(max(0, -o), n - max(0, o)), slice(max(0, o), n - max(0, -o))
                (sz, tz), (sy, ty), (sx, tx) = sl(0, dz, Z), sl(0, dy, Y), sl(0, dx, X)
                same = L[sz, sy, sx] == L[tz, ty, tx]
                inside = Tc[c - 1][sz, sy, sx] < Dl[tz, ty, tx]
                covered[sz, sy, sx] |= same & inside
    kept = obj & ~covered
    work = int(Nt[Dl][kept].sum())
    return work, int(kept.sum())


def copy_calibration(dev, nbytes: int = 1 << 30):
    """One plain device copy of a known size, so that the HBM counters of a profiled
    run can be scaled: bytes / FETCH_SIZE and bytes / WRITE_SIZE of this copy."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    print(f"# copy calibration: {nbytes} bytes read and written", flush=True)


# Source files that define each kernel family; a recorded HBM-counter figure is used
# only while these files (comments and blank space removed) are unchanged.
KERNEL_SOURCES = {
    "edt": ("paper_2504_05808_amd/csrc/edt.hip", "paper_2504_05808_amd/csrc/lt_internal.h"),
    "thickness": ("paper_2504_05808_amd/csrc/thickness.hip", "paper_2504_05808_amd/csrc/lt_internal.h"),
    "measures": ("paper_2504_05808_amd/csrc/measures.hip", "paper_2504_05808_amd/csrc/lt_internal.h"),
}
KERNEL_FAMILY = {"edt_pass_x": "edt", "edt_pass_y": "edt", "edt_pass_z": "edt", "bbox_runs": "thickness",
                 "prune3d": "thickness", "fronts3d": "thickness", "paint_tiles": "thickness",
                 "object_sums": "measures"}
COUNTERS_FILE = os.path.join(ROOT, "profiles", "hbm_counters_512cube.json")


def source_digest(family: str) -> str:
    import hashlib
    import re
    h = hashlib.sha1()
    for rel in KERNEL_SOURCES[family]:
        text = open(os.path.join(ROOT, rel)).read()
        text = re.sub(r"//[^\n]*", "", text)
        h.update(re.sub(r"\s+", "", text).encode())
    return h.hexdigest()[:16]


def recorded_traffic(kernel: str):
    """HBM bytes per launch from the recorded FETCH_SIZE / WRITE_SIZE runs, scaled by
    the copy calibration, or None when absent or taken on other kernel sources."""
    fam = KERNEL_FAMILY.get(kernel)
    if fam is None or not os.path.exists(COUNTERS_FILE):
        return None
    rec = json.load(open(COUNTERS_FILE))
    k = rec.get("kernels", {}).get(kernel)
    if not k or rec.get("source_digest", {}).get(fam) != source_digest(fam):
        return None
    cal = rec["calibration"]
    return k["fetch_kib"] * 1024 * cal["fetch_scale"] + k["write_kib"] * 1024 * cal["write_scale"]


def _cpu_leg(vol, boxes, order, seconds: float, threads: int) -> dict:
    """Oracle on per-object crops of the objects in `order` for about `seconds`,
    `threads` objects at a time; per-stage times are summed over the objects."""
    from concurrent.futures import ThreadPoolExecutor

    from oracle import lt_oracle as O

    def one(l):
        box = boxes[int(l)]
        lo = [max(0, a - 1) for a in box[0]]
        hi = [min(n, b + 1) for b, n in zip(box[1], vol.shape)]
        sub = (vol[tuple(slice(a, b) for a, b in zip(lo, hi))] == l).astype(np.int64)
        t0 = time.perf_counter()
        d = O.edt_sq(sub)
        t1 = time.perf_counter()
        lt = O.local_thickness_sq(d)
        t2 = time.perf_counter()
        sums = O.object_sums(sub, lt, 1)
        O.closed_forms(sums, 3)
        t3 = time.perf_counter()
        return int(sub.sum()), t1 - t0, t2 - t1, t3 - t2

    done, vox, stage = 0, 0, np.zeros(3)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        i = 0
        while time.perf_counter() - t0 < seconds and i < len(order):
            batch = order[i:i + threads]
            i += len(batch)
            for v, a, b, c in ex.map(one, batch):
                done += 1
                vox += v
                stage += (a, b, c)
    return dict(done=done, vox=vox, seconds=time.perf_counter() - t0, stage=stage)


def cpu_baseline(vol: np.ndarray, seconds: float, threads: int, single_seconds: float) -> dict:
    """The CPU oracle (per-object crops, exact D and LT in C, FP64 measures in
    numpy) on bounded random samples of the volume's objects: one leg with
    `threads` objects in flight, one single-threaded leg on other objects."""
    from oracle import lt_oracle as O

    boxes = O.object_boxes(vol)
    labels = np.array(sorted(boxes))
    order = np.random.default_rng(0).permutation(labels)
    multi = _cpu_leg(vol, boxes, order, seconds, threads)
    single = _cpu_leg(vol, boxes, order[multi["done"]:], single_seconds, 1) if single_seconds > 0 else None

    def rates(leg):
        frac = leg["done"] / len(labels)
        return vol.size * frac / leg["seconds"], leg["done"] / leg["seconds"]

    v, o = rates(multi)
    out = {
        "value": float(v),
        "unit": "voxels/s",
        "objects_per_s": o,
        "cores": threads,
        "kind": "oracle",
        "sample": f"{multi['done']} of {len(labels)} objects (random order), {multi['seconds']:.1f} s, "
                  f"{threads} objects at a time, per-object crops; voxels/s = volume voxels x sampled "
                  f"object fraction / time",
        "stage_share": {k: round(float(x / multi["stage"].sum()), 4)
                        for k, x in zip(("edt", "thickness", "measures"), multi["stage"])},
    }
    if single is not None and single["done"]:
        sv, so = rates(single)
        out["single_thread"] = {
            "value": float(sv), "unit": "voxels/s", "objects_per_s": so, "cores": 1,
            "sample": f"{single['done']} further objects, {single['seconds']:.1f} s",
            "stage_s_per_object": {k: round(float(x / single["done"]), 5)
                                   for k, x in zip(("edt", "thickness", "measures"), single["stage"])},
        }
    return out


def batch_bench(args):
    """Batched form vs plain per-volume launches on the same GPU: 64 uint16 cubes
    with edges U{96..384} and U{10..500} objects each (half ellipsoids, half
    superellipsoids of the 512^3 distribution; ``--batch-reduced``: edges U{64..160},
    U{5..60} objects)."""
    import torch

    from paper_2504_05808_amd import lt, synth

    n = args.batch_volumes
    edges, counts = ((64, 160), (5, 60)) if args.batch_reduced else ((96, 384), (10, 500))
    t0 = time.perf_counter()
    vols = synth.cfg4_batch(n_volumes=n, edges=edges, counts=counts)
    print(f"# batch of {n} volumes generated in {time.perf_counter() - t0:.1f}s", flush=True)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ctx = lt.default_context()
    labs = [torch.from_numpy(v).to(dev) for v in vols]
    mls = [int(v.max()) for v in vols]
    vox = sum(v.size for v in vols)
    objs = sum(mls)
    b = lt.Batch(list(zip(labs, mls)), ctx=ctx,
                 autotune_cache=os.environ.get("LT_AUTOTUNE_CACHE"), autotune_repeats=2)
    plain_out = [(torch.empty(l.shape, dtype=torch.int32, device=dev),
                  torch.empty(l.shape, dtype=torch.int32, device=dev),
                  lt.alloc_measures(ml + 1, dev)) for l, ml in zip(labs, mls)]

    def plain():
        for l, ml, (d, t, m) in zip(labs, mls, plain_out):
            lt.edt(l, out=d, ctx=ctx)
            lt.thickness(l, d, ml, out=t, ctx=ctx)
            lt.object_measures(l, t, ml, out=m, ctx=ctx)

    def fused():                                    # the same kernels as the graph, one stream
        for l, ml, out in zip(labs, mls, plain_out):
            lt.pipeline(l, ml, out=out, ctx=ctx)

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        z = torch.cuda.Event(enable_timing=True)
        t_host = time.perf_counter()
        a.record()
        for _ in range(args.steps):
            fn()
        z.record()
        torch.cuda.synchronize()
        return a.elapsed_time(z) / args.steps, (time.perf_counter() - t_host) * 1e3 / args.steps

    ms_plain, host_plain = timed(plain)
    ms_fused, host_fused = timed(fused)
    ms_graph, host_graph = timed(b.run)
    ctx.sync_status()
    status = b.status()
    same = all(torch.equal(p[1], q[1]) for p, q in zip(plain_out, b.outputs))
    # share of the voxels that lie in some object's bounding box (the rest is
    # background that the streaming passes still read)
    from scipy import ndimage
    boxed = 0
    for v in vols:
        mask = np.zeros(v.shape, bool)
        for sl in ndimage.find_objects(v.astype(np.int32)):
            if sl is not None:
                mask[sl] = True
        boxed += int(mask.sum())
    print(json.dumps({
        "metric": "batched volumes: voxels/s, one graph launch vs per-volume plain launches",
        "value": vox / (ms_graph * 1e-3), "unit": "voxels/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_graph, "higher_is_better": True,
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"{n} uint16 cubes, edges {edges[0]}-{edges[1]}, "
                               f"{counts[0]}-{counts[1]} objects each", "voxels": vox, "objects": objs},
        "plain_three_calls": {"ms_per_step": ms_plain, "host_ms_per_step": host_plain,
                              "voxels_per_s": vox / (ms_plain * 1e-3)},
        "plain_fused": {"ms_per_step": ms_fused, "host_ms_per_step": host_fused,
                        "voxels_per_s": vox / (ms_fused * 1e-3)},
        "graph": {"ms_per_step": ms_graph, "host_ms_per_step": host_graph,
                  "objects_per_s": objs / (ms_graph * 1e-3)},
        "speedup_vs_three_calls": ms_plain / ms_graph, "speedup_vs_fused": ms_fused / ms_graph,
        "boxed_voxel_share": boxed / vox, "volume_status": status,
        "identical_lt": bool(same), "tuning": ctx.get_tuning(),
    }), flush=True)
    b.close()


MLP_FWD_FLOPS = 2 * (34 * 64 + 64 * 64 + 64 * 64 + 64)     # per object, unpadded layer sizes
BF16_PEAK_TFLOPS = 2500.0


def mlp_bench(args):
    """Learned correction on its own: AdamW training steps (batch 256) and corrected
    sphericity for 20000 objects (the evaluation volume's object count), synthetic
    features; one line with both rates."""
    import torch

    from paper_2504_05808_amd import lt

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ctx = lt.default_context()
    g = torch.Generator().manual_seed(0)
    n_obj, B = 20000, 256
    x = torch.rand((n_obj, 34), generator=g).to(dev)
    y = torch.randn(n_obj, generator=g).to(dev)
    s_lt = (0.7 + 0.3 * torch.rand(n_obj, generator=g)).to(dev)
    net = lt.MLP(seed=0, ctx=ctx)
    batches = [(x[i:i + B].contiguous(), y[i:i + B].contiguous()) for i in range(0, n_obj - B + 1, B)]

    def timed(fn, k):
        for i in range(args.warmup):
            fn(i)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        z = torch.cuda.Event(enable_timing=True)
        a.record()
        for i in range(k):
            fn(i)
        z.record()
        torch.cuda.synchronize()
        return a.elapsed_time(z) / k

    n_train = max(args.steps, 50)
    train = lambda i: net.train_step(*batches[i % len(batches)], lr=1e-3, weight_decay=1e-4)
    correct = lambda i: net.correct(x, s_lt)
    ms_train = timed(train, n_train)                      # clean timing, no per-kernel events
    ms_corr = timed(correct, args.steps)
    # second pass with the library's per-launch events: the kernel breakdown
    ctx.profile(True)
    ctx.profile_reset()
    for i in range(n_train):
        train(i)
    torch.cuda.synchronize()
    prof_train = ctx.profile_read()
    ctx.profile_reset()
    for i in range(args.steps):
        correct(i)
    torch.cuda.synchronize()
    prof_corr = ctx.profile_read()
    ctx.profile(False)
    ctx.sync_status()
    launches_per_step = sum(v[1] for v in prof_train.values()) / n_train
    train_flops = 3 * MLP_FWD_FLOPS * B
    infer_flops = MLP_FWD_FLOPS * n_obj
    roof = None
    fb = prof_train.get("mlp_fused_fwd_bwd")
    if fb:
        ach = n_train * train_flops / (fb[0] * 1e-3) / 1e12
        roof = {"bound": "mfma", "kernel": "mlp_fused_fwd_bwd", "achieved": round(ach, 4), "peak": BF16_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(ach / BF16_PEAK_TFLOPS, 6), "traffic": None,
                "avg_ms": round(fb[0] / fb[1], 5), "launches": fb[1],
                "note": "algorithmic products of a training step (unpadded 34-64-64-64-1, backward = 2x "
                        "forward) over the fused kernel's time; latency-bound at these sizes"}
    inf = prof_corr.get("mlp_fused_infer")
    print(json.dumps({
        "metric": "learned correction: corrected sphericities per second and training samples per second",
        "value": n_obj / (ms_corr * 1e-3), "unit": "objects/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_corr, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "34-64-64-64-1 SiLU MLP, 20000 objects per correction call, "
                               "AdamW batch 256"},
        "train": {"ms_per_step": ms_train, "samples_per_s": B / (ms_train * 1e-3),
                  "launches_per_step": launches_per_step,
                  "kernel_ms": {k: round(v[0] / v[1], 5) for k, v in prof_train.items()}},
        "correct": {"kernel_ms": {k: round(v[0] / v[1], 5) for k, v in prof_corr.items()},
                    "infer_tflops": None if not inf else round(
                        args.steps * infer_flops / (inf[0] * 1e-3) / 1e12, 4)},
        "roofline": roof,
    }), flush=True)
    net.close()


def extensions_bench(ctx, lab, dist_sq, lt_sq, max_label: int, reps: int = 10, large: bool = True) -> dict:
    """The calls beyond the step, each timed alone on the resident volume (outside
    the step's timed region): kernel times from the library's per-launch HIP events
    and algorithmic GB/s against the HBM peak."""
    import torch

    from paper_2504_05808_amd import lt
    N = lab.numel()
    lb = lab.element_size()
    out = {}

    def timed(name, fn, kernel_bytes_map):
        fn()
        ctx.sync_status()
        ctx.profile(True)
        ctx.profile_reset()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        prof = ctx.profile_read()
        ctx.profile(False)
        ctx.sync_status()
        ks = {k: v[0] / v[1] for k, v in prof.items()}
        rec = {"ms": round(sum(v[0] for v in prof.values()) / reps, 4),
               "kernel_ms": {k: round(v, 4) for k, v in ks.items()}}
        for k, b in kernel_bytes_map.items():
            if k in ks:
                gbs = b / (ks[k] * 1e-3) / 1e9
                rec.setdefault("kernel_GBs", {})[k] = round(gbs, 1)
                rec.setdefault("hbm_frac", {})[k] = round(gbs / HBM_PEAK_GBS, 4)
        out[name] = rec

    # mesh-based surface measures: one streaming read of the labels
    timed("mesh_measures", lambda: lt.mesh_measures(lab, max_label, ctx=ctx),
          {"mesh_area3d": lb * N})
    # anisotropic spacing: the volume sampled every second slice (256 x 512 x 512,
    # slices twice as thick as pixels: squared spacings 4, 1, 1), the whole path
    lab_a = lab[::2].contiguous()
    Na = lab_a.numel()
    out_a = (torch.empty_like(lab_a, dtype=torch.int32), torch.empty_like(lab_a, dtype=torch.int32),
             lt.alloc_measures(max_label + 1, lab.device))
    timed("pipeline_aniso_4_1_1", lambda: lt.pipeline_aniso(lab_a, max_label, (4, 1, 1), out=out_a, ctx=ctx), {})
    rec = out["pipeline_aniso_4_1_1"]
    rec["workload"] = "512^3 volume, every second slice: 256 x 512 x 512 uint16, squared spacings (4, 1, 1)"
    rec["voxels_per_s"] = Na / (rec["ms"] * 1e-3)
    rec["pipeline_hbm_frac"] = round(36.0 * Na / (rec["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    del out_a, lab_a
    # large objects (the banded paint launch): one digital ball of radius 150 (D up to
    # 22,501) and one noisy superellipsoid grain with semi-axes 150 x 120 x 97.5, each
    # alone in a 512^3 volume -- the large-radius end of the EDT searches and ball cover
    from paper_2504_05808_amd import synth
    large_objects = ()
    if large:
        rng = synth.rng_for(9150)
        grain, _ = synth.superellipsoid_mask((150.0, 120.0, 97.5), 0.7, 0.9, synth.haar_rotation(rng), 3.0, rng)
        large_objects = (("pipeline_ball_r150", synth.ball_mask(150)[0], "one digital ball of radius 150"),
                         ("pipeline_grain_150", grain,
                          "one noisy superellipsoid grain, semi-axes 150 x 120 x 97.5 (Haar rotation)"))
    for name, obj, what in large_objects:
        big = np.zeros(tuple(lab.shape), np.uint16)
        o = [(n - b) // 2 for n, b in zip(big.shape, obj.shape)]
        big[o[0]:o[0] + obj.shape[0], o[1]:o[1] + obj.shape[1], o[2]:o[2] + obj.shape[2]] = obj
        big_t = torch.from_numpy(big).to(lab.device)
        out_b = (torch.empty_like(big_t, dtype=torch.int32), torch.empty_like(big_t, dtype=torch.int32),
                 lt.alloc_measures(2, lab.device))
        timed(name, lambda: lt.pipeline(big_t, 1, out=out_b, ctx=ctx), {})
        out[name]["workload"] = f"{what} ({int(obj.sum())} voxels) in a 512^3 uint16 volume"
        out[name]["voxels_per_s"] = float(obj.sum()) / (out[name]["ms"] * 1e-3)
        del out_b, big_t, big
    # roughness-filtered roundness, half-width 2: three separable window passes
    # (x: labels, D, LT -> F; y: labels, F -> F; z: labels, F, D, LT -> per-label sums)
    timed("filtered_roundness_w2", lambda: lt.filtered_roundness(lab, dist_sq, lt_sq, max_label, 2, ctx=ctx),
          {"rough_x": (lb + 12) * N, "rough_y": (lb + 8) * N, "rough_z_final": (lb + 12) * N})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--cpu-single-seconds", type=float, default=8.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch", action="store_true",
                    help="measure the batched graph form against per-volume launches instead")
    ap.add_argument("--batch-volumes", type=int, default=64)
    ap.add_argument("--batch-reduced", action="store_true",
                    help="batch of smaller cubes (edges 64-160, 5-60 objects) that builds in seconds")
    ap.add_argument("--mlp", action="store_true", help="measure the learned correction instead")
    ap.add_argument("--autotune", action="store_true",
                    help="let the library's autotuner choose the kernel knobs first (outside the timed region)")
    ap.add_argument("--paint-rows", type=int, default=0, help="paint tile rows (32 or 64; 0 = default)")
    ap.add_argument("--paint-per-cu", type=int, default=0, help="paint blocks per CU (1 or 2; 0 = default)")
    ap.add_argument("--front-chunk", type=int, default=0, help="z-front chunk (32, 64, 128; 0 = default)")
    ap.add_argument("--no-large", action="store_true",
                    help="leave out the large-object calls (profiled runs: their empty launches of the "
                         "plain paint kernel would enter its per-dispatch averages)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 1 GiB device copy first (reference for the HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the path shards by "
              "independent objects, and this benchmark measures one GPU's throughput.", file=sys.stderr)
        sys.exit(2)
    if args.batch:
        batch_bench(args)
        return
    if args.mlp:
        mlp_bench(args)
        return

    import torch

    from paper_2504_05808_amd import lt, synth

    t_gen = time.perf_counter()
    vol, meta = synth.cfg3()
    t_gen = time.perf_counter() - t_gen
    n_obj = int(meta["n_objects"])
    max_label = int(vol.max())
    N = vol.size
    f_obj = float((vol != 0).mean())
    print(f"# workload 512^3 uint16 objects={n_obj} fill={f_obj:.3f} gen={t_gen:.1f}s", flush=True)

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    lab = torch.from_numpy(vol).to(dev)
    ctx = lt.default_context()
    d = torch.empty(vol.shape, dtype=torch.int32, device=dev)
    t = torch.empty(vol.shape, dtype=torch.int32, device=dev)
    m = lt.alloc_measures(max_label + 1, dev)

    knobs = {k: v for k, v in (("paint_tile_rows", args.paint_rows), ("paint_blocks_per_cu", args.paint_per_cu),
                               ("front_chunk", args.front_chunk)) if v}
    if knobs:
        ctx.set_tuning(**knobs)
    if args.autotune:
        t_at = time.perf_counter()
        ctx.autotune(lab, max_label, cache_path=os.environ.get("LT_AUTOTUNE_CACHE"), repeats=2)
        print(f"# autotune {time.perf_counter() - t_at:.1f}s -> {ctx.get_tuning()}", flush=True)
    print(f"# device {ctx.info()} tuning {ctx.get_tuning()}", flush=True)
    if args.copy_calibration:
        copy_calibration(dev)

    def step():
        lt.pipeline(lab, max_label, out=(d, t, m), ctx=ctx)

    for _ in range(args.warmup):
        step()
    ctx.sync_status()
    print("# warmup done", flush=True)

    # timed region: the steps alone, no per-kernel instrumentation
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(args.steps):
        step()
    stop.record()
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(stop)
    ctx.sync_status()
    ms = total_ms / args.steps

    # second pass over as many steps: every kernel bracketed by HIP events recorded
    # on its launch stream (the library's profiler), for the per-kernel breakdown
    ctx.profile(True)
    ctx.profile_reset()
    torch.cuda.synchronize()
    start.record()
    for _ in range(args.steps):
        step()
    stop.record()
    torch.cuda.synchronize()
    prof_ms = start.elapsed_time(stop) / args.steps
    prof = ctx.profile_read()
    ctx.profile(False)
    ctx.sync_status()

    kernels = {k: {"avg_ms": v[0] / v[1], "launches": v[1]} for k, v in prof.items()}
    dom = max(kernels, key=lambda k: kernels[k]["avg_ms"] * kernels[k]["launches"])
    dom_ms = kernels[dom]["avg_ms"]
    for k, v in kernels.items():
        b = kernel_bytes(k, N, f_obj)
        if b is not None:
            v["GBs"] = b / (v["avg_ms"] * 1e-3) / 1e9
    roof = None
    work = kept = None
    if dom == "paint_tiles":
        work, kept = ball_cover_work(lab, d)
        ops = 2.0 * work                             # a compare and a max per covered point
        ach = ops / (dom_ms * 1e-3) / 1e12
        roof = {"bound": "alu", "kernel": dom, "achieved": round(ach, 3), "peak": round(ALU_PEAK_TOPS, 2),
                "unit": "Tops/s", "frac": round(ach / ALU_PEAK_TOPS, 4), "traffic": recorded_traffic(dom),
                "work_per_launch": ops, "avg_ms": round(dom_ms, 4),
                "note": "ball-cover work: 2 x sum over kept centres of |B(x)| (compare + max per "
                        "covered lattice point) / kernel time; peak = 32-bit VALU lanes x clock"}
    else:
        b = kernel_bytes(dom, N, f_obj)
        if b is not None:
            ach = b / (dom_ms * 1e-3) / 1e9
            roof = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": recorded_traffic(dom),
                    "bytes_per_launch": b, "avg_ms": round(dom_ms, 4)}
    stage = {"edt": 0.0, "thickness": 0.0, "measures": 0.0}
    for k, v in kernels.items():
        tot = v["avg_ms"] * v["launches"] / args.steps
        if k.startswith("edt"):
            stage["edt"] += tot
        elif k in ("object_sums", "zero_measure_arrays", "closed_forms", "lt_histogram"):
            stage["measures"] += tot
        else:
            stage["thickness"] += tot
    pipe_bytes = 36.0 * N
    pipe_gbs = pipe_bytes / (ms * 1e-3) / 1e9

    ext = extensions_bench(ctx, lab, d, t, max_label, large=not args.no_large)

    cpu = None
    if not args.no_cpu_baseline:
        # the host share of one GPU on the test machines is 16 cores
        threads = min(16, len(os.sched_getaffinity(0)))
        cpu = cpu_baseline(vol, args.cpu_seconds, threads, args.cpu_single_seconds)

    out = {
        "metric": METRIC,
        "value": N / (ms * 1e-3),
        "unit": "voxels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "512^3 uint16 label volume, superellipsoids with value-noise "
                               "surfaces (semi-axes 4-30), exact EDT + local thickness + measures",
                   "voxels": N, "objects": n_obj, "fill": round(f_obj, 4)},
        "objects_per_s": n_obj / (ms * 1e-3),
        "profiled_ms_per_step": round(prof_ms, 4),
        "roofline": roof,
        "pipeline_hbm": {"bytes_per_step": pipe_bytes, "achieved_GBs": round(pipe_gbs, 1),
                         "frac": round(pipe_gbs / HBM_PEAK_GBS, 4),
                         "note": "36 B/voxel pass-structured algorithmic traffic / step time"},
        "stage_ms": {k: round(v, 4) for k, v in stage.items()},
        "device": ctx.info(),
        "tuning": ctx.get_tuning(),
        "kernel_ms": {k: round(v["avg_ms"], 4) for k, v in kernels.items()},
        "kernel_GBs": {k: round(v["GBs"], 1) for k, v in kernels.items() if "GBs" in v},
        "ball_cover": None if work is None else {"work_points": work, "kept_centres": kept,
                                                 "points_per_object_voxel": work / (f_obj * N)},
        "extensions": ext,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
