"""Benchmark of the gfx950 adaptive AD-census matcher.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-extras]
                    [--extras staged,batched,soft] [--cpu-rows N]

A step is one pass of the whole plain matcher (census and arms of both views,
cost and two-stage aggregation of both views, WTA with sub-pixel refinement,
LR check) over one 1280x720 pair with D = 128, through the one-call entry
point ``dco_stereo_match``.  Inputs are resident in HBM before timing starts.
The JSON line carries:
  value        Mpix*disp/s = W*H*D / seconds per step / 1e6
  roofline     the dominant kernel (largest share of the step) against its
               bound, with its duration from HIP events recorded by the
               library on its own stream over a second pass of the timed
               steps (the events stay out of the headline loop)
  cpu_baseline the CPU oracle (single thread) on a bounded sample of the
               same pair
  extras       stage times, the median / p90 of single-step times, and
               (with --extras, default on) the staged four-call path per
               stage against the HBM roofline and the other paths
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
# One CDNA4 compute unit issues one 64-lane VALU instruction per SIMD per
# 4 cycles (16 lanes per cycle each): 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz.
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
METRIC = "Mpix·disp/s and ms/frame at 1280x720 D=128 vs oracle; batched & fwd+bwd vs plain"
STAGES = ("census+arms+counts", "cost+aggregate L+R", "wta", "lrcheck", "vote")


TRAFFIC_PROFILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                               "plain_match_1280x720_D128_hbm_counters.md")


SQ_PROFILE = os.path.join(os.path.dirname(TRAFFIC_PROFILE),
                          "plain_match_1280x720_D128_sq_counters.md")


def _profile_fields(path, keys):
    """The `key: value` lines of a committed counter summary, or None when the
    dominant kernel's sources have changed since those counters were taken."""
    import hashlib
    try:
        fields = dict(l.split(": ", 1) for l in open(path).read().splitlines()
                      if l.startswith(tuple(keys) + ("kernel_source",)))
        h = hashlib.sha256()
        for s in fields["kernel_sources"].split():
            h.update(open(os.path.join(os.path.dirname(path), "..", s), "rb").read())
        if h.hexdigest() != fields["kernel_source_sha256"].strip():
            return None
        return {k: fields[k].strip() for k in keys}
    except (OSError, KeyError, ValueError):
        return None


def measured_traffic():
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when the
    kernel's sources have changed since those counters were taken."""
    f = _profile_fields(TRAFFIC_PROFILE, ["traffic_bytes_per_launch"])
    return int(f["traffic_bytes_per_launch"]) if f else None


def measured_frame_traffic():
    """HBM bytes of one whole one-call frame (FETCH_SIZE + WRITE_SIZE of
    every kernel of the step, copy-calibrated) from the committed counter
    summary, or None when a kernel of the step has changed since."""
    f = _profile_fields(TRAFFIC_PROFILE, ["frame_traffic_bytes"])
    return int(f["frame_traffic_bytes"]) if f else None


def measured_busy():
    """Busy fractions of the dominant kernel's VALU, TA, TD and LDS from the
    committed SQ/TA/TD counter summary (same validity rule as the traffic)."""
    keys = ["busy_valu", "busy_ta", "busy_td", "busy_lds", "valu_lane_ops_per_pd"]
    f = _profile_fields(SQ_PROFILE, keys)
    return {k.replace("busy_", ""): float(v) for k, v in f.items()} if f else None


def step_distribution(m, gL, gR, disp, valid, steps):
    """Median and 90th percentile of single-step times (HIP events on the
    stream the matcher runs on), measured after the timed loop."""
    import torch
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    for a, b in ev:
        a.record()
        m.match(gL, gR, disp, valid)
        b.record()
    torch.cuda.synchronize()
    t = np.sort([a.elapsed_time(b) for a, b in ev])
    return dict(median=round(float(np.median(t)), 4),
                p90=round(float(t[min(len(t) - 1, int(np.ceil(0.9 * len(t))) - 1)]), 4),
                min=round(float(t[0]), 4), n=len(t))


def _guarded(fn, *args):
    """Run one extra measurement; a Python-level failure is recorded in its
    place so that the headline line is still printed."""
    try:
        return fn(*args)
    except Exception as e:  # noqa: BLE001 - reported, not hidden
        log(f"bench: {fn.__name__} failed: {e!r}")
        return {"error": repr(e)}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(L, R, D, rows):
    """The oracle on the first `rows` rows of the pair (single thread)."""
    import oracle
    H, W = L.shape[:2]
    t0 = time.perf_counter()
    oracle.match(L[:rows], R[:rows], D)
    dt = time.perf_counter() - t0
    units = W * rows * D
    return dict(value=units / dt / 1e6, unit="Mpix·disp/s", cores=1, kind="oracle",
                sample=f"rows 0..{rows - 1} of the {W}x{H} D={D} pair ({rows}/{H} of the frame), "
                       f"whole plain matcher, {dt:.1f} s")


# Rows of context a band needs so that its rows equal the whole-frame
# result: 2 L1 for the two vertical aggregation stages, plus L1 for the
# vertical arms of the pixels in those ranges (which also covers the census
# window's 3 rows).
BAND_HALO = 51


def oracle_bands(L, R, D, nbands, threads):
    """The oracle over the whole frame in `nbands` row bands run on `threads`
    threads at once (the oracle's C calls release the GIL).  Each band is
    matched with BAND_HALO rows of context on each side; its own rows of the
    result are exactly the whole-frame result.  Returns (disp, valid, seconds,
    rows matched in all)."""
    import concurrent.futures as cf
    import oracle
    H, W = L.shape[:2]
    edges = np.linspace(0, H, nbands + 1).round().astype(int)
    disp = np.empty((H, W), np.float32)
    valid = np.empty((H, W), np.uint8)

    def run(i):
        y0, y1 = int(edges[i]), int(edges[i + 1])
        a, b = max(0, y0 - BAND_HALO), min(H, y1 + BAND_HALO)
        d, v, _, _ = oracle.match(L[a:b], R[a:b], D)
        disp[y0:y1] = d[y0 - a:y1 - a]
        valid[y0:y1] = v[y0 - a:y1 - a]

    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(threads) as ex:
        list(ex.map(run, range(nbands)))
    dt = time.perf_counter() - t0
    rows = sum(min(H, int(edges[i + 1]) + BAND_HALO) - max(0, int(edges[i]) - BAND_HALO)
               for i in range(nbands))
    return disp, valid, dt, rows


def cpu_all_cores(L, R, D):
    """Second CPU figure: the same oracle on every host core the process may
    use (at most 16), over the whole frame in row bands.  Returns the figure
    and the oracle's (disp, valid) of the whole frame."""
    n = min(16, len(os.sched_getaffinity(0)))
    H, W = L.shape[:2]
    disp, valid, dt, rows = oracle_bands(L, R, D, n, n)
    return dict(value=W * H * D / dt / 1e6, unit="Mpix·disp/s", cores=n,
                kind="oracle, row bands on threads",
                sample=f"whole {W}x{H} D={D} frame in {n} bands with a {BAND_HALO}-row halo "
                       f"({rows} rows matched in all), {dt:.1f} s"), disp, valid


def accuracy_gate(disp, valid, odisp, ovalid):
    """The timed step's output against the oracle's whole frame, bit for bit."""
    bad_v = int(np.count_nonzero(valid != ovalid))
    bad_d = int(np.count_nonzero(disp.view(np.uint32) != odisp.astype(np.float32).view(np.uint32)))
    return dict(bit_exact=bad_v == 0 and bad_d == 0, mismatched_valid=bad_v,
                mismatched_disp=bad_d, pixels=int(valid.size),
                valid_frac=round(float(ovalid.mean()), 4),
                compared="every pixel of disp (float bits) and valid of the timed step's "
                         "output against the oracle's whole frame")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=540)
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--extras", default="staged,sizes,vote,half,densify,contour,batched,soft",
                    help="comma list of the extra measurements to run "
                         "(staged, sizes, vote, half, densify, contour, batched, soft)")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MiB",
                    help="only run a plain device copy of MiB mebibytes (counter calibration)")
    args = ap.parse_args()
    want = set() if args.no_extras else {e for e in args.extras.split(",") if e}
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(pairs would shard across GPUs with no communication); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2203_02300_amd import StereoMatcher, synth
    from paper_2203_02300_amd._lib import check, lib

    if args.copy_calib:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE readings
        # scale the same counters of the matcher's kernels
        n = args.copy_calib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": n * 4, "calls": 3}), flush=True)
        return

    W, H, D = 1280, 720, 128
    log("bench: generating the 1280x720 D=128 pair (seed 3)")
    pair = synth.config_c3()
    L, R = pair["left"], pair["right"]
    gL = torch.from_numpy(L).cuda()
    gR = torch.from_numpy(R).cuda()
    m = StereoMatcher(W, H, D)
    disp = torch.empty((H, W), dtype=torch.float32, device="cuda")
    valid = torch.empty((H, W), dtype=torch.uint8, device="cuda")
    for _ in range(args.warmup):
        m.match(gL, gR, disp, valid)
    torch.cuda.synchronize()
    log(f"bench: warmup done, timing {args.steps} steps")

    t0 = time.perf_counter()
    for _ in range(args.steps):
        m.match(gL, gR, disp, valid)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    # Stage times come from a second pass of the same steps with the
    # library's per-stage HIP events on its stream: ten event records per
    # step cost ~0.05 ms, so they stay out of the headline loop.
    log("bench: timing the stages (library HIP events)")
    check(lib().dco_stereo_profile(m._h, 1))
    for _ in range(args.steps):
        m.match(gL, gR, disp, valid)
    torch.cuda.synchronize()
    check(lib().dco_stereo_profile(m._h, 0))
    stage_ms = (C.c_float * len(STAGES))()
    calls = C.c_int()
    check(lib().dco_stereo_stage_times(m._h, stage_ms, len(STAGES), C.byref(calls)))
    per_call = [stage_ms[i] / calls.value for i in range(len(STAGES))]
    log("bench: stage ms " + ", ".join(f"{n}={t:.4f}" for n, t in zip(STAGES, per_call)))

    units = W * H * D
    value = units / (ms_step / 1e3) / 1e6
    P, V = W * H, W * H * D
    # dominant kernel: cost + two-stage aggregation of both views (one launch)
    agg_ms = per_call[1]
    # algorithmic VALU work of the launch: ~14 ops for the raw cost and ~26
    # for the four range sums and two divisions per (p, d), for 2 V entries
    ops_per_unit = 40
    achieved = ops_per_unit * 2 * V / (agg_ms / 1e3) / 1e12
    # the whole step against HBM: the staged path's algorithmic bytes
    # (32 V + 99 P, what the four-call chain must move) and the bytes the
    # one-call step measurably moves (all of its kernels, counters)
    staged_bytes = 32 * V + 99 * P
    frame_bytes = measured_frame_traffic()
    step_s = ms_step / 1e3
    hbm = dict(staged_algorithmic_bytes=staged_bytes,
               staged_bytes_frac=round(staged_bytes / step_s / 1e9 / HBM_PEAK_GBS, 4),
               measured_frame_bytes=frame_bytes,
               measured_frame_frac=(round(frame_bytes / step_s / 1e9 / HBM_PEAK_GBS, 4)
                                    if frame_bytes else None),
               peak_GBs=HBM_PEAK_GBS)
    roofline = dict(bound="alu", achieved=round(achieved, 2), peak=round(VALU_PEAK_TOPS, 2),
                    unit="TOP/s", frac=round(achieved / VALU_PEAK_TOPS, 4), traffic=measured_traffic(),
                    kernel="k_agg_pair_ws", kernel_ms=round(agg_ms, 4),
                    ops_per_pd=ops_per_unit, units_per_launch=2 * V,
                    units_busy=measured_busy(), hbm_step=hbm)

    head_disp, head_valid = disp.cpu().numpy(), valid.cpu().numpy()
    extras = {"stage_ms": {n: round(t, 4) for n, t in zip(STAGES, per_call)},
              "step_ms": step_distribution(m, gL, gR, disp, valid, args.steps)}
    if "staged" in want:
        extras["staged"] = _guarded(staged_extras, m, gL, gR, args.steps)
    if "sizes" in want:
        log("bench: one-call match at 64x48 D=16 and 640x480 D=64")
        extras["sizes"] = _guarded(sizes_extras, args.steps)
    if "vote" in want:
        log("bench: one-call match with two Eq. 4 vote passes")
        extras["vote"] = _guarded(vote_extras, gL, gR, disp, valid, args.steps)
    if "half" in want:
        log("bench: quarter-size front end (640x360, D=64, two vote passes, depth)")
        extras["half"] = _guarded(half_extras, gL, gR, args.steps)
    if "contour" in want:
        log("bench: depth contour filter (1280x720 frame, 640x360 flows)")
        extras["contour"] = _guarded(contour_extras, args.steps)
    if "densify" in want:
        log("bench: depth densification (Eq. 13-20) at 640x360 and 1280x720")
        extras["densify"] = _guarded(densify_extras, max(3, args.steps // 10))
    del m
    torch.cuda.empty_cache()
    if "batched" in want:
        log("bench: batched matcher (32 mixed pairs)")
        extras["batched"] = _guarded(batched_extras, max(3, args.steps // 10))
        torch.cuda.empty_cache()
    if "soft" in want:
        log("bench: differentiable soft-argmin (8 x 640x480, D=64)")
        extras["soft"] = _guarded(soft_extras, max(3, args.steps // 10))
        torch.cuda.empty_cache()

    cpu = None
    accuracy = dict(bit_exact=None, compared="not run (--no-cpu)")
    if not args.no_cpu:
        log(f"bench: CPU oracle on {args.cpu_rows} rows")
        cpu = cpu_baseline(L, R, D, args.cpu_rows)
        if "sizes" in want:
            log("bench: CPU oracle at 64x48 D=16 and 640x480 D=64 (whole frames, one thread)")
            extras["sizes_oracle"] = _guarded(sizes_oracle)
        log("bench: CPU oracle on all cores (row bands)")
        res = _guarded(cpu_all_cores, L, R, D)
        if isinstance(res, tuple):
            extras["cpu_all_cores"], odisp, ovalid = res
            accuracy = accuracy_gate(head_disp, head_valid, odisp, ovalid)
            log(f"bench: accuracy gate bit_exact={accuracy['bit_exact']}")
        else:
            extras["cpu_all_cores"] = res

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "Mpix·disp/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32 (Q20 fixed point) + f32",
        "data": "synthetic",
        "config": {"workload": "plain matcher, one 1280x720 RGB pair, D=128, 10 slanted planes "
                               "+ 2 boxes, noise 2, right gain 0.9..1.1 (seed 3)",
                   "W": W, "H": H, "D": D, "entry": "dco_stereo_match"},
        "bit_exact": accuracy["bit_exact"], "accuracy": accuracy,
        "roofline": roofline, "cpu_baseline": cpu, "extras": extras,
    }
    print(json.dumps(out), flush=True)


def _time(fn, n):
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(n):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / n


def batched_extras(n):
    """32 pairs of mixed size and disparity range: one graph launch per batch,
    against the same pairs matched one by one with dco_stereo_match."""
    import torch
    from paper_2203_02300_amd import BatchMatcher, StereoMatcher, synth
    pairs = synth.config_c4()
    shapes = [(p["W"], p["H"], p["D"]) for p in pairs]
    Ls = [torch.from_numpy(p["left"]).cuda() for p in pairs]
    Rs = [torch.from_numpy(p["right"]).cuda() for p in pairs]
    units = sum(W * H * D for W, H, D in shapes)
    t0 = time.perf_counter()
    bm = BatchMatcher(shapes)
    create_s = time.perf_counter() - t0
    disps = [torch.empty((H, W), device="cuda") for W, H, D in shapes]
    valids = [torch.empty((H, W), dtype=torch.uint8, device="cuda") for W, H, D in shapes]
    ms_batch = _time(lambda: bm.match(Ls, Rs, disps, valids), n)
    tiles = [bm.tile(i) for i in range(len(shapes))]
    bm.close()
    ms_plain = 0.0
    same = True
    for i, (W, H, D) in enumerate(shapes):
        with StereoMatcher(W, H, D) as m:
            d, v = m.match(Ls[i], Rs[i])
            ms_plain += _time(lambda: m.match(Ls[i], Rs[i], d, v), 2)
            same &= bool(torch.equal(d, disps[i]) and torch.equal(v, valids[i]))
    return dict(pairs=len(shapes), sum_WHD=units, ms_per_batch=round(ms_batch, 3),
                ms_per_pair=round(ms_batch / len(shapes), 4),
                Mpix_disp_s=round(units / (ms_batch / 1e3) / 1e6, 1),
                plain_ms_sum=round(ms_plain, 3),
                plain_Mpix_disp_s=round(units / (ms_plain / 1e3) / 1e6, 1),
                speedup_vs_plain=round(ms_plain / ms_batch, 3), bit_identical_to_plain=same,
                create_s=round(create_s, 2),
                tiles_band_dchunk=sorted(set((t[1], t[2]) for t in tiles)))


def soft_extras(n):
    """Forward + backward of the soft-argmin head (8 pairs, 640x480, D=64)
    against the plain matcher on the same 8 pairs."""
    import torch
    from paper_2203_02300_amd import StereoMatcher, synth
    from paper_2203_02300_amd.soft import soft_argmin_disparity
    pairs = synth.config_c5()
    W, H, D = 640, 480, 64
    L = torch.from_numpy(np.stack([p["left"] for p in pairs])).cuda()
    R = torch.from_numpy(np.stack([p["right"] for p in pairs])).cuda()
    gt = torch.from_numpy(np.stack([p["disp"] for p in pairs])).cuda()
    mask = ~torch.from_numpy(np.stack([p["occluded"] for p in pairs])).cuda()
    theta = torch.tensor([10.0, 30.0, 1.0], device="cuda", requires_grad=True)  # initial theta of the differentiable workload
    m = StereoMatcher(W, H, D)

    def step():
        theta.grad = None
        dhat = soft_argmin_disparity(m, L, R, theta)
        loss = ((dhat - gt).abs() * mask).sum() / mask.sum()
        loss.backward()
        return loss

    ms_fb = _time(step, n)
    loss = float(step())
    grad = theta.grad.detach().cpu().tolist()
    ms_plain = _time(lambda: [m.match(L[b], R[b]) for b in range(L.shape[0])], n)
    m.close()
    units = L.shape[0] * W * H * D
    return dict(pairs=int(L.shape[0]), ms_fwd_bwd=round(ms_fb, 3),
                Mpix_disp_s=round(units / (ms_fb / 1e3) / 1e6, 1),
                plain_ms=round(ms_plain, 3), ratio_to_plain=round(ms_fb / ms_plain, 3),
                loss=round(loss, 4), grad_theta=[round(g, 6) for g in grad])


def sizes_extras(steps):
    """The one-call match on the two smaller workloads (64x48 with D = 16,
    launch-bound; 640x480 with D = 64): ms per frame and Mpix*disp/s."""
    import torch
    from paper_2203_02300_amd import StereoMatcher, synth
    out = {}
    for name, pair, D in (("64x48 D=16", synth.config_c1(), 16),
                          ("640x480 D=64", synth.config_c2(), 64)):
        L = torch.from_numpy(pair["left"]).cuda()
        R = torch.from_numpy(pair["right"]).cuda()
        H, W = L.shape[:2]
        m = StereoMatcher(W, H, D)
        disp = torch.empty((H, W), dtype=torch.float32, device="cuda")
        valid = torch.empty((H, W), dtype=torch.uint8, device="cuda")
        ms = _time(lambda: m.match(L, R, disp, valid), steps)
        m.close()
        out[name] = dict(ms_per_frame=round(ms, 4), Mpix_disp_s=round(W * H * D / ms / 1e3, 1))
    return out


def sizes_oracle():
    """CPU leg at the two smaller workloads: the oracle on one thread over the
    whole frame (timed), and the one-call match's maps against it, bit for
    bit."""
    import torch
    import oracle
    from paper_2203_02300_amd import StereoMatcher, synth
    out = {}
    for name, pair, D in (("64x48 D=16", synth.config_c1(), 16),
                          ("640x480 D=64", synth.config_c2(), 64)):
        H, W = pair["left"].shape[:2]
        with StereoMatcher(W, H, D) as m:
            disp, valid = m.match(torch.from_numpy(pair["left"]).cuda(),
                                  torch.from_numpy(pair["right"]).cuda())
            torch.cuda.synchronize()
            gdisp, gvalid = disp.cpu().numpy(), valid.cpu().numpy()
        t0 = time.perf_counter()
        odisp, ovalid, _, _ = oracle.match(pair["left"], pair["right"], D)
        dt = time.perf_counter() - t0
        gate = accuracy_gate(gdisp, gvalid, ovalid=ovalid, odisp=odisp)
        out[name] = dict(oracle_ms_1thread=round(dt * 1e3, 1),
                         oracle_Mpix_disp_s=round(W * H * D / dt / 1e6, 2),
                         bit_exact=gate["bit_exact"], mismatched_disp=gate["mismatched_disp"],
                         mismatched_valid=gate["mismatched_valid"])
    return out


def vote_extras(gL, gR, disp0, valid0, steps):
    """The one-call match with two passes of the Eq. 4 region vote on the
    same pair: ms per frame, the vote stage's HIP-event time, and how many
    valid pixels the vote changed."""
    import torch
    from paper_2203_02300_amd import StereoMatcher
    from paper_2203_02300_amd._lib import check, lib
    H, W = gL.shape[:2]
    m = StereoMatcher(W, H, 128, vote_iters=2)
    disp = torch.empty_like(disp0)
    valid = torch.empty_like(valid0)
    ms = _time(lambda: m.match(gL, gR, disp, valid), steps)
    check(lib().dco_stereo_profile(m._h, 1))
    for _ in range(steps):
        m.match(gL, gR, disp, valid)
    torch.cuda.synchronize()
    check(lib().dco_stereo_profile(m._h, 0))
    st = (C.c_float * len(STAGES))()
    calls = C.c_int()
    check(lib().dco_stereo_stage_times(m._h, st, len(STAGES), C.byref(calls)))
    m.close()
    changed = int(((disp != disp0) & (valid == 1)).sum())
    return dict(passes=2, ms_per_frame=round(ms, 4), vote_stage_ms=round(st[4] / calls.value, 4),
                Mpix_disp_s=round(W * H * 128 / (ms / 1e3) / 1e6, 1),
                valid_pixels=int(valid.sum()), changed_pixels=changed)


def half_extras(gL, gR, steps):
    """The paper's operating point: the 1280x720 pair reduced to 640x360,
    matched with D = 64 and two Eq. 4 vote passes, disparity doubled and
    converted to depth, all on the GPU: ms per frame."""
    import torch
    from paper_2203_02300_amd import StereoMatcher
    H2, W2 = gL.shape[:2]
    W, H, D = W2 // 2, H2 // 2, 64
    m = StereoMatcher(W, H, D, vote_iters=2)
    ms = _time(lambda: m.match_half(gL, gR, 1000.0), steps)
    _, valid, _ = m.match_half(gL, gR, 1000.0)
    torch.cuda.synchronize()
    m.close()
    return dict(full=f"{W2}x{H2}", reduced=f"{W}x{H}", D=D, vote_passes=2,
                ms_per_frame=round(ms, 4), valid_frac=round(float(valid.float().mean()), 4))


def contour_extras(steps):
    """The depth contour filter of Sec. 5 on a seeded 1280x720 frame with
    flows on the 640x360 grid: ms per frame and hysteresis launches."""
    import torch
    from paper_2203_02300_amd import ContourFilter, synth
    d = synth.contour_inputs(1280, 720, 11)
    t = {k: torch.from_numpy(d[k]).cuda() for k in ("rgb", "past", "future")}
    f = ContourFilter(1280, 720)
    ms = _time(lambda: f.run(t["rgb"], t["past"], t["future"]), steps)
    B, _, _ = f.run(t["rgb"], t["past"], t["future"])
    out = dict(ms_per_frame=round(ms, 4), hysteresis_launches=f.launches(),
               contour_frac=round(float(B.float().mean()), 4))
    f.close()
    return out


def densify_extras(n):
    """Depth densification (Eq. 13-20) on seeded synthetic inputs at the
    paper's reduced grid and at the full frame: ms per solve, iterations, and
    the iteration kernels' HBM rate for their algorithmic bytes (per pixel
    and iteration: 7 FP64 reads and 2 writes in the direction launch, 5 reads
    and 2 writes in the update launch, neighbours counted once)."""
    import torch
    from paper_2203_02300_amd import Densifier, synth
    out = {}
    for W, H in ((640, 360), (1280, 720)):
        d = synth.densify_inputs(W, H, 7)
        t = {k: torch.from_numpy(d[k]).cuda() for k in ("Ds", "Dpre", "Bdp", "Mfuse", "MI")}
        z = Densifier(W, H)
        run = lambda: z.run(t["Ds"], t["Bdp"], t["Mfuse"], t["MI"], Dpre=t["Dpre"])
        ms = _time(run, n)
        it, rel = z.stats()
        z.close()
        bytes_iter = (9 + 7) * 8 * W * H
        out[f"{W}x{H}"] = dict(ms_per_solve=round(ms, 3), iterations=it, rel_residual=rel,
                               us_per_iteration=round(ms * 1e3 / max(it, 1), 2),
                               GBs_iteration_bytes=round(bytes_iter * it / (ms / 1e3) / 1e9, 1))
    return out


def staged_extras(m, gL, gR, steps):
    """Per-stage times of the four-call path, against the HBM roofline."""
    import torch
    W, H, D = m.W, m.H, m.D
    P, V = W * H, W * H * D
    cL, aL = m.census(gL)
    cR, aR = m.census(gR)
    costL = m.cost_volume(0, gL, gR, cL, cR, aL)
    costR = m.cost_volume(1, gL, gR, cL, cR, aR)
    aggL = m.aggregate(costL, aL)
    aggR = m.aggregate(costR, aR)
    torch.cuda.synchronize()
    n = max(3, steps // 5)
    # algorithmic bytes per call (each stage reads its inputs and writes its outputs once)
    stages = {
        "census": (lambda: (m.census(gL), m.census(gR)), 2 * (3 * P + 8 * P + 4 * P)),
        "cost_volume": (lambda: (m.cost_volume(0, gL, gR, cL, cR, aL, costL),
                                 m.cost_volume(1, gL, gR, cL, cR, aR, costR)),
                        2 * (4 * V + 3 * P * 2 + 8 * P * 2 + 4 * P)),
        "aggregate": (lambda: (m.aggregate(costL, aL, aggL), m.aggregate(costR, aR, aggR)),
                      2 * (8 * V + 4 * P)),
        "wta_lrcheck": (lambda: m.wta_lrcheck(aggL, aggR), 8 * V + 9 * P),
    }
    res = {}
    total = 0.0
    for name, (fn, nbytes) in stages.items():
        fn()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(n):
            fn()
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / n
        total += ms
        gbs = nbytes / (ms / 1e3) / 1e9
        res[name] = dict(ms=round(ms, 4), GBs=round(gbs, 1), hbm_frac=round(gbs / HBM_PEAK_GBS, 4),
                         bytes=nbytes)
    allbytes = sum(b for _, b in stages.values())
    res["total"] = dict(ms=round(total, 4), GBs=round(allbytes / (total / 1e3) / 1e9, 1),
                        hbm_frac=round(allbytes / (total / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                        Mpix_disp_s=round(V / (total / 1e3) / 1e6, 1))
    del costL, costR, aggL, aggR
    return res


if __name__ == "__main__":
    main()
