"""Benchmark: particle updates/s of the SIR filter step on one MI355X.

Workload (default): one spot tracked through 1024x1024 fp32 frames with
N = 38,000,000 particles, spot width s = 2 px, 13x13 likelihood patch,
systematic resampling every step (the paper's 38-million-particle case on a
single GPU). A step is one frame: gather + propagate + patch likelihood +
normalisation/ESS + resampling for all N particles. Frames are synthetic
(paper_1310_5045_amd.synth) and resident on the GPU before timing starts;
filter initialisation is outside the timed region.

Prints one JSON line. `value` is N * steps / GPU time of the timed steps
(two HIP events on the filter's stream around them).

No figure is printed (exit status 3) when the filter's output fails a check:
after the timed steps the final ESS, the tracking error, the normalisation,
ESS and estimate against the particles' own weights, and the resampling
invariants of the last step are checked on the GPU's output; the
cpu_baseline leg then runs one more step and checks it against the oracle on
sampled particles (propagation, log weights, every ancestor). The same
workload is also timed from the other initial cloud (`init_alternative`:
stratified when the headline uses the uniform cloud, uniform otherwise). The
uniform cloud is the paper's (i.i.d. uniform draws, Section 6.3) with the
particles placed in the Z order of their draws, so that a workgroup's 256
particles are neighbours in the image from the first frame on.
`roofline` covers the dominant kernel (k_step) against the fp64 vector peak;
`roofline_resample` covers the ancestor passes against HBM bandwidth; both
use algorithmic work per launch / average launch time measured with HIP
events on the filter's stream. `cpu_baseline` times the FP64 oracle on a
bounded sample of the same workload on the host.

`roofline.traffic` is the HBM traffic of one k_step launch in bytes, taken
from two rocprofv3 counter runs (FETCH_SIZE, then WRITE_SIZE) of this script
with `--copy-probe-mib` and a fixed `--shape`, each counter scaled by what it
reads for a plain device copy of known size. The step kernel's workgroup
shapes differ in traffic (one may spill registers to scratch memory), so each
shape has its own record: `--traffic-from FETCH_DB WRITE_DB --shape S` turns
the two databases into profiles/traffic_k_step_shape<S>_<workload>.json,
stamped with a hash of the kernel sources; a run reports the record of the
shape its steps ran with, while the hash still matches (null otherwise).
"""
import argparse
import glob
import hashlib
import json
import os
import sqlite3
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6
KERNEL_SOURCES = ("paper_1310_5045_amd/csrc/ppf_kernels.hip",
                  "paper_1310_5045_amd/csrc/ppf_internal.hpp")


def kernel_source_hash():
    """sha256 of the kernel sources' code: comments, trailing blanks and empty
    lines removed, so that only a change of the code itself invalidates a
    traffic record (the sources hold no string literal with a comment
    marker)."""
    import re
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        lines = [re.sub(r"//.*$", "", ln).rstrip() for ln in text.split("\n")]
        h.update("\n".join(ln for ln in lines if ln).encode())
    return h.hexdigest()


def traffic_path(kernel, workload, shape):
    tag = f"_shape{shape}" if shape is not None else ""
    return os.path.join(ROOT, "profiles", f"traffic_{kernel}{tag}_{workload}.json")


def _counter_per_dispatch(db, counter):
    """{dispatch_id: (kernel name, counter summed over the dispatch's instances)}."""
    con = sqlite3.connect(db)
    rows = con.execute("select dispatch_id, kernel_name, counter_name, sum(value) "
                       "from counters_collection group by dispatch_id, counter_name").fetchall()
    con.close()
    return {d: (k, v) for d, k, c, v in rows if c == counter}


# Kernel groups with traffic records: the kernel names a group's dispatches
# carry, and whether the record depends on the step kernel's workgroup shape.
TRAFFIC_GROUPS = {
    "k_step": dict(match=("k_step_spot",), per_shape=True),
    # the resampling pair: the ancestor pass and its long-run fill, per step
    "k_resample": dict(match=("k_anc", "k_fill"), per_shape=False),
    # a batch's step launches: the fused one and the wide-patch one, per step
    # (counter runs with --shape 1: one fused launch per step)
    "k_step_batch": dict(match=("k_step_batch_fused", "k_step_batch_wide"), per_shape=False),
}


def traffic_from(fetch_db, write_db, workload, copy_mib, warmup, steps, shape, kernel="k_step"):
    """Writes the traffic record of kernel group `kernel` (TRAFFIC_GROUPS)
    from a FETCH_SIZE and a WRITE_SIZE counter database of `bench.py
    --copy-probe-mib copy_mib --shape shape` runs with the given warm-up and
    timed steps: each counter's average over the timed launches (the last
    `steps` dispatches of each kernel of the group, summed over the group's
    kernels), scaled by what the counter reads for the device copy of
    copy_mib MiB."""
    grp = TRAFFIC_GROUPS[kernel]
    copy_bytes = copy_mib * (1 << 20)
    per = {}
    for name, db in (("FETCH_SIZE", fetch_db), ("WRITE_SIZE", write_db)):
        d = _counter_per_dispatch(db, name)
        avg_kib, launches = 0.0, {}
        for match in grp["match"]:
            names = [d[i][0] for i in sorted(d) if match in d[i][0]]
            ker = [d[i][1] for i in sorted(d) if match in d[i][0]]
            if grp["per_shape"]:
                # k_step_spot<P, S>: the timed launches must all be of shape S
                tag = f", {shape}>"
                if not names or any(tag not in nm for nm in names[-steps:]):
                    raise SystemExit(f"{db}: the timed {match} launches are not all of shape "
                                     f"{shape}")
            if len(ker) < steps + warmup:
                raise SystemExit(f"{db}: {len(ker)} {match} dispatches, expected at least "
                                 f"{steps + warmup}")
            ker = ker[-steps:]
            avg_kib += sum(ker) / len(ker)
            launches[match] = len(ker)
        # the probe copies copy_bytes: the largest reading among the kernels
        # named like a copy
        cp = ([v for k, v in d.values() if "copy" in k.lower()] or
              [v for k, v in d.values() if "elementwise" in k.lower()])
        if not cp:
            raise SystemExit(f"{db}: no copy dispatches with {name}")
        kib_copy = max(cp)
        per[name] = dict(kernel_kib_avg=avg_kib, launches=launches, copy_kib=kib_copy,
                         scale=copy_bytes / (kib_copy * 1024.0))
    traffic = sum(per[c]["kernel_kib_avg"] * 1024.0 * per[c]["scale"] for c in per)
    shp = shape if grp["per_shape"] else None
    rec = {"kernel": kernel, "shape": shp, "workload": workload,
           "source_sha256": kernel_source_hash(),
           "traffic_bytes_per_launch": traffic, "copy_probe_bytes": copy_bytes,
           "counters": per,
           "command": [f"rocprofv3 --kernel-trace --pmc {c} -d <dir> -o run -- python3 bench.py "
                       f"--steps {steps} --warmup {warmup} --no-cpu-baseline --no-alt-init "
                       f"--copy-probe-mib {copy_mib} --shape {shape}" for c in per]}
    with open(traffic_path(kernel, workload, shp), "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    return rec


def load_traffic(kernel, workload, shape):
    """Bytes per launch of a traffic record, while its kernel sources match
    (None otherwise)."""
    shp = shape if TRAFFIC_GROUPS[kernel]["per_shape"] else None
    try:
        with open(traffic_path(kernel, workload, shp)) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != kernel_source_hash():
        return None
    return rec["traffic_bytes_per_launch"]


WORKLOADS = {
    # frame size, frames, particles, spot width, patch, resampling threshold
    "sir_1024x1024_n38m_p13": dict(W=1024, H=1024, T=20, n=38_000_000, s=2.0, P=13,
                                   thr=float("inf")),
    "sir_512x512_n1m_p9": dict(W=512, H=512, T=50, n=1 << 20, s=1.5, P=9, thr=float(1 << 19)),
    # the same with the distributed schemes over groups of 256 (4096 groups)
    "rna_512x512_n1m_p9": dict(W=512, H=512, T=50, n=1 << 20, s=1.5, P=9, thr=float(1 << 19),
                               scheme=(1, 256, 0)),
    "arna_512x512_n1m_p9": dict(W=512, H=512, T=50, n=1 << 20, s=1.5, P=9, thr=float(1 << 19),
                                scheme=(3, 256, 0), rho=0.5, rho_min=0.05),
    "rpa_gs_512x512_n1m_p9": dict(W=512, H=512, T=50, n=1 << 20, s=1.5, P=9,
                                  thr=float(1 << 19), scheme=(2, 256, 0)),
    "rpa_sgs_512x512_n1m_p9": dict(W=512, H=512, T=50, n=1 << 20, s=1.5, P=9,
                                   thr=float(1 << 19), scheme=(2, 256, 1)),
    # the 38M workload with RPA over groups of 250 (152,000 groups; 38 M is
    # not a multiple of 256)
    "rpa_gs_1024x1024_n38m_p13": dict(W=1024, H=1024, T=20, n=38_000_000, s=2.0, P=13,
                                      thr=float("inf"), scheme=(2, 250, 0)),
    "rpa_sgs_1024x1024_n38m_p13": dict(W=1024, H=1024, T=20, n=38_000_000, s=2.0, P=13,
                                       thr=float("inf"), scheme=(2, 250, 1)),
    "sir_128x128_n4096_p9": dict(W=128, H=128, T=10, n=4096, s=1.5, P=9, thr=float("inf")),
    # forward pass with the derivatives of log p^ in (s, b, sigma, q, I0)
    # (the cloud starts within 5 px of the spot: at I = 25 and s = 1.7 a cloud
    # spread over the frame locks onto empty patches, where low-intensity
    # particles explain the pixels as well as the spot's own do)
    "grad_512x512_n262k_p11": dict(W=512, H=512, T=30, n=1 << 18, s=1.7, P=11, thr=float("inf"),
                                   I=25.0, grad=1, init_radius=5.0),
    "grad_1024x1024_n38m_p13": dict(W=1024, H=1024, T=20, n=38_000_000, s=2.0, P=13,
                                    thr=float("inf"), grad=1),
    # 256 spots, one independent filter each, stepped as one batch
    "multitrack_1024x1024_t256": dict(W=1024, H=1024, T=30, tracks=256, n_lo=1024, n_hi=262144,
                                      s_lo=1.2, s_hi=2.5, I_lo=15.0, I_hi=60.0, vmax=2.0,
                                      thr=float("inf")),
}


def multitrack_setup(ppf, synth, w):
    """The multi-spot movie and one filter per spot: N_t log-uniform in
    [n_lo, n_hi], the spot's own PSF width (patch 2 floor(3 s) + 1), an init
    box of +-5 px around the spot's first position, velocities in
    [-vmax, vmax], intensity within a factor 2 of the spot's."""
    import numpy as np
    mv = synth.render_movie(w["W"], w["H"], w["T"], n_spots=w["tracks"],
                            intensity=(w["I_lo"], w["I_hi"]), sigma=(w["s_lo"], w["s_hi"]),
                            vmax=w["vmax"], start_box=(0, w["W"], 0, w["H"]), seed=1)
    rng = np.random.default_rng(1)
    ns = np.rint(np.exp(rng.uniform(np.log(w["n_lo"]), np.log(w["n_hi"]), w["tracks"])))
    ps = []
    for t in range(w["tracks"]):
        x0, y0 = mv.truth[0, t]
        I = float(mv.intensity[t])
        ps.append(ppf.params(n_particles=int(ns[t]), width=w["W"], height=w["H"],
                             psf_sigma=float(mv.sigma[t]), background=10.0, noise_sigma=3.0,
                             init_a=(x0 - 5, y0 - 5, -w["vmax"], -w["vmax"], I / 2),
                             init_b=(x0 + 5, y0 + 5, w["vmax"], w["vmax"], 1.5 * I),
                             ess_threshold=w["thr"], seed=1, track_id=t))
    return mv, ps


def run_multitrack(args, w):
    import math

    import numpy as np
    import torch

    import paper_1310_5045_amd as ppf
    from paper_1310_5045_amd import synth

    mv, ps = multitrack_setup(ppf, synth, w)
    K, Wm = args.steps, args.warmup
    T = w["T"]
    torch.cuda.set_device(0)
    frames = torch.from_numpy(mv.frames).cuda()
    if args.copy_probe_mib:
        src = torch.ones(args.copy_probe_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    b = ppf.Batch(ps)
    graph = args.launch == "graph"
    gpu_ms, wall, kt, tuned, _ = timed_steps(torch, b, frames, K, Wm, T, graph, args.shape)
    sts = b.stats()
    ntot = sum(int(p.n_particles) for p in ps)
    flops = sum(4 * ppf.patch_size(p) ** 2 * int(p.n_particles) for p in ps)
    step_ms = kt.get("k_step", (0, 0.0))[1] / K
    achieved_tf = flops / (step_ms / 1e3) / 1e12 if step_ms > 0 else 0.0
    err = [float(np.linalg.norm(sts[t]["mean"][:2] - mv.truth[(K - 1) % T, t]))
           for t in range(len(ps))]
    # a lost track may end with all its weight on one particle (ESS = 1)
    bad = [t for t in range(len(ps))
           if not (math.isfinite(sts[t]["ess"]) and sts[t]["ess"] >= 1.0 - 1e-9)]
    if bad:
        raise GateError(f"tracks {bad[:8]} end with ESS < 1 or not finite")
    if not float(np.median(err)) <= 1.0:
        raise GateError(f"median tracking error {np.median(err):.3f} px")
    out = {
        "metric": "particle updates/s, 256 independent tracks batched on 1 GPU",
        "value": ntot * K / (gpu_ms / 1e3),
        "unit": "particle updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": gpu_ms / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 state, f64 likelihood/normalisation",
        "data": "synthetic",
        "config": {"workload": args.workload, "tracks": len(ps), "n_particles_total": ntot,
                   "n_min": min(int(p.n_particles) for p in ps),
                   "n_max": max(int(p.n_particles) for p in ps),
                   "patches": sorted({ppf.patch_size(p) for p in ps}),
                   "frame": [w["W"], w["H"]], "resampling": "systematic", "frames_timed": K,
                   "launch": args.launch, "autotune": tuned},
        "roofline": {"bound": "alu", "kernel": "k_step (all patch sizes)",
                     "achieved": achieved_tf, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved_tf / FP64_VECTOR_PEAK_TFLOPS,
                     "traffic": load_traffic("k_step_batch", args.workload, None),
                     "step_kernels_ms_per_step": step_ms},
        "kernel_ms_total": {k: v[1] for k, v in kt.items()},
        "kernel_launches": {k: v[0] for k, v in kt.items()},
        "wall_s": wall,
        "tracking_error_px_median": float(np.median(err)),
        "checks": "passed",
    }
    b.close()
    del b
    # plain SIR on the same GPU (the 38M single-filter workload), for the ratio
    pw = WORKLOADS["sir_1024x1024_n38m_p13"]
    pmv = synth.render_movie(pw["W"], pw["H"], pw["T"], intensity=30.0, sigma=pw["s"],
                             background=10.0, noise_sd=3.0, seed=1)
    pframes = torch.from_numpy(pmv.frames).cuda()
    pf = ppf.Filter(make_params(ppf, pw, ppf.INIT_UNIFORM_ZORDER))
    pms, _, _, _, _ = timed_steps(torch, pf, pframes, K, Wm, pw["T"], False, None)
    check_state(ppf, pf, pw, pmv, (K - 1) % pw["T"], 0)
    pf.close()
    plain = pw["n"] * K / (pms / 1e3)
    out["plain_sir"] = {"workload": "sir_1024x1024_n38m_p13", "value": plain,
                        "ms_per_step": pms / K}
    out["ratio_to_plain"] = out["value"] / plain
    print(json.dumps(out), flush=True)


# The differentiable-SIR experiment: 512 x 512, T = 30, N = 262,144, P = 11,
# one spot rendered with s = 1.7, I = 25, b = 10, sigma_xi = 3 and a truth
# that follows the filter's own motion model (position, velocity and
# intensity random walks with the sds q), so that every parameter of theta
# has a generating value; the start point moves each by 20 % (I0, the offset
# of the initial intensity range, by 20 % of I).
C5 = dict(W=512, H=512, T=30, n=1 << 18, P=11, s=1.7, I=25.0, b=10.0, sigma=3.0,
          q=(0.5, 0.5, 0.1, 0.1, 1.0), movie_seed=5, filter_seed=1,
          start=(1.2, 0.8, 1.2, 0.8, 1.2, 0.8, 1.2, 0.8), I0_start=0.2)


def c5_setup(ppf, synth):
    """(movie, base params at the generating theta, theta_true, theta_start)
    of the differentiable-SIR experiment; the initial cloud covers +-5 px
    around the spot's first position, velocities in [-1, 1], intensities in
    [I/2, 3 I/2] (+ I0)."""
    c = C5
    mv = synth.render_movie(c["W"], c["H"], c["T"], intensity=c["I"], sigma=c["s"],
                            background=c["b"], noise_sd=c["sigma"], jitter=c["q"][0],
                            vel_jitter=c["q"][2], int_jitter=c["q"][4], seed=c["movie_seed"])
    x0, y0 = mv.truth[0, 0]
    base = ppf.params(n_particles=c["n"], width=c["W"], height=c["H"], psf_sigma=c["s"],
                      patch=c["P"], background=c["b"], noise_sigma=c["sigma"], q=c["q"],
                      init_a=(x0 - 5, y0 - 5, -1, -1, c["I"] / 2),
                      init_b=(x0 + 5, y0 + 5, 1, 1, 1.5 * c["I"]),
                      ess_threshold=float("inf"), seed=c["filter_seed"])
    true = [float(v) for v in ppf.theta_of(base)]
    start = [t * f for t, f in zip(true[:8], c["start"])] + [c["I0_start"] * c["I"]]
    return mv, base, true, start


def grad_run(ppf, p, frames, means=None):
    """One run of the filter p (gradient mode) over frames: (log p^, d log p^
    / d theta, the ancestors of every step); `means` (a list) receives each
    step's MMSE estimate."""
    import numpy as np
    f = ppf.Filter(p)
    ancs = []
    for k in range(frames.shape[0]):
        f.step(frames[k])
        ancs.append(f.particles()[2])
        if means is not None:
            means.append(np.asarray(f.stats()["mean"], dtype=np.float64))
    cum, _ = f.loglik()
    g, _ = f.grad()
    f.close()
    return cum, np.asarray(g, dtype=np.float64), np.stack(ancs)


def replay_run(ppf, p, frames, ancs, centres=None):
    """log p^ of the filter p over frames with the given ancestors instead of
    its own: after each step the resampled cloud x~_k[anc_k] is set back with
    log weights -log N, so the next step propagates particle i from it with
    its own Philox draws, as the recorded run did. `centres` (a list)
    receives each step's patch centres round(x~), (2, N) int32."""
    import math

    import numpy as np
    n = int(p.n_particles)
    q = ppf.Params.from_buffer_copy(p)
    q.grad = 0
    f = ppf.Filter(q)
    lw = np.full(n, -math.log(n))
    for k in range(frames.shape[0]):
        f.step(frames[k])
        if k + 1 < frames.shape[0] or centres is not None:
            x, _, _ = f.particles()
            if centres is not None:
                centres.append(np.floor(x[:2].astype(np.float64) + 0.5).astype(np.int32))
            if k + 1 < frames.shape[0]:
                f.set_particles(np.ascontiguousarray(x[:, ancs[k]]), lw)
    cum, _ = f.loglik()
    f.close()
    return cum


def run_grad_check(args):
    """The differentiable-SIR experiment on the GPU: the derivatives at the
    start point against central differences of log p^ with the start point's
    ancestors replayed (h = 1e-3 of each parameter, of I for I0), then 50
    Adam steps of gradient ascent from the start point (in log theta for the
    positive parameters, in I0 / I for I0)."""
    import math

    import numpy as np
    import torch

    import paper_1310_5045_amd as ppf
    from paper_1310_5045_amd import synth

    torch.cuda.set_device(0)
    mv, base, true, start = c5_setup(ppf, synth)
    frames = torch.from_numpy(mv.frames).cuda()
    c = C5
    p0 = ppf.params_at(base, start)
    cum0, g0, ancs = grad_run(ppf, p0, frames)
    rep0 = replay_run(ppf, p0, frames, ancs)
    names = list(ppf.GRAD_NAMES)
    fd, moved = [], []
    for j in range(9):
        h = 1e-3 * (abs(start[j]) if j < 8 else c["I"])
        tp = list(start)
        tm = list(start)
        tp[j] += h
        tm[j] -= h
        cp, cm = [], []
        lp = replay_run(ppf, ppf.params_at(base, tp), frames, ancs, cp)
        lm = replay_run(ppf, ppf.params_at(base, tm), frames, ancs, cm)
        fd.append((lp - lm) / (2 * h))
        # particle-steps whose patch centre differs between the two runs
        moved.append(int(sum(int(np.sum(np.any(a != b, axis=0))) for a, b in zip(cp, cm))))
        print(f"fd {names[j]}: {fd[-1]:.6g} (gradient {g0[j]:.6g}, {moved[-1]} patches moved)",
              file=sys.stderr, flush=True)
        del cp, cm
    fd = np.array(fd)
    # ascent: u_j = log theta_j (j < 8), u_8 = I0 / I
    scale = np.array([1.0] * 8 + [c["I"]])

    def to_u(th):
        return np.array([math.log(v) for v in th[:8]] + [th[8] / c["I"]])

    def to_theta(u):
        return [math.exp(v) for v in u[:8]] + [u[8] * c["I"]]

    u = to_u(start)
    m1 = np.zeros(9)
    m2 = np.zeros(9)
    lr, b1, b2 = 0.03, 0.9, 0.999
    trace = []
    for it in range(1, args.ascent_steps + 1):
        th = to_theta(u)
        L, g, _ = grad_run(ppf, ppf.params_at(base, th), frames)
        du = np.array([th[j] * g[j] for j in range(8)] + [g[8] * scale[8]])
        trace.append({"step": it - 1, "theta": th, "loglik": L})
        m1 = b1 * m1 + (1 - b1) * du
        m2 = b2 * m2 + (1 - b2) * du * du
        step = lr * (0.95 ** (it - 1)) * (m1 / (1 - b1 ** it)) / (np.sqrt(m2 / (1 - b2 ** it)) + 1e-12)
        u = u + step
        print(f"ascent {it - 1}: L {L:.3f} theta {np.round(th, 4).tolist()}", file=sys.stderr,
              flush=True)
    th_end = to_theta(u)
    mean_end, mean_true, mean_start = [], [], []
    L_end, _, _ = grad_run(ppf, ppf.params_at(base, th_end), frames, mean_end)
    trace.append({"step": args.ascent_steps, "theta": th_end, "loglik": L_end})
    L_true, _, _ = grad_run(ppf, ppf.params_at(base, true), frames, mean_true)
    grad_run(ppf, p0, frames, mean_start)

    def track_err(means):
        """RMS over the frames of the MMSE estimate's error in position (px)
        and in intensity against the generator's truth."""
        mm = np.stack(means)
        dp = mm[:, :2] - mv.truth[:, 0]
        dI = mm[:, 4] - mv.intensity_track[:, 0]
        return {"position_px": float(np.sqrt(np.mean(np.sum(dp * dp, axis=1)))),
                "intensity": float(np.sqrt(np.mean(dI * dI)))}
    rel = np.abs(fd - g0) / np.maximum(np.abs(g0), 1e-12)
    out = {
        "experiment": "differentiable SIR: d log p^ / d theta, central differences, ascent",
        "config": {"workload": "grad_c5_512x512_n262k_p11", "n_particles": c["n"],
                   "frame": [c["W"], c["H"]], "frames": c["T"], "patch": c["P"],
                   "generator": {"s": c["s"], "I": c["I"], "b": c["b"], "sigma": c["sigma"],
                                 "q": list(c["q"]), "seed": c["movie_seed"]},
                   "resampling": "systematic every step, ancestors held fixed in the derivative"},
        "theta_names": names,
        "theta_true": true,
        "theta_start": start,
        "start": {"loglik": cum0, "gradient": g0.tolist(), "central_difference": fd.tolist(),
                  "fd_h": [1e-3 * (abs(start[j]) if j < 8 else c["I"]) for j in range(9)],
                  "rel_diff": rel.tolist(), "patches_moved_between_runs": moved,
                  "particle_steps": c["n"] * c["T"],
                  "replay_loglik_minus_run": rep0 - cum0},
        "ascent": {"method": f"Adam, lr {lr} x 0.95^t, {args.ascent_steps} steps, log theta "
                             "(I0 / I for I0)",
                   "trace": trace, "theta_end": th_end, "loglik_end": L_end,
                   "loglik_at_theta_true": L_true,
                   "rel_error_start": [abs(a - b) / abs(b) if b else abs(a) / c["I"]
                                       for a, b in zip(start, true)],
                   "rel_error_end": [abs(a - b) / abs(b) if b else abs(a) / c["I"]
                                     for a, b in zip(th_end, true)],
                   "tracking_rms": {"start": track_err(mean_start), "end": track_err(mean_end),
                                    "true": track_err(mean_true)}},
    }
    print(json.dumps(out), flush=True)


# --init: the library's init kind of each initial cloud
INIT_KINDS = {"uniform": lambda ppf: ppf.INIT_UNIFORM_ZORDER,
              "stratified": lambda ppf: ppf.INIT_STRATIFIED,
              "uniform-unordered": lambda ppf: ppf.INIT_UNIFORM}


def make_params(ppf, w, init_kind, grad=0):
    """The filter of a single-filter workload: the initial cloud covers the
    spot's start box (default the whole frame), intensity within a factor
    of 2 of the spot's."""
    x0, x1, y0, y1 = w.get("box", (0, w["W"], 0, w["H"]))
    I = w.get("I", 30.0)
    resample, group, dlb = w.get("scheme", (0, 256, 0))
    return ppf.params(n_particles=w["n"], width=w["W"], height=w["H"], psf_sigma=w["s"],
                      background=10.0, noise_sigma=3.0, patch=w["P"], init_kind=init_kind,
                      init_a=(x0, y0, -1, -1, I / 2), init_b=(x1, y1, 1, 1, 1.5 * I),
                      ess_threshold=w["thr"], seed=1, grad=grad, resample=resample,
                      rna_group=group, dlb=dlb, rna_exchange=w.get("rho", 0.1),
                      arna_min=w.get("rho_min", 0.0))


def timed_steps(torch, f, frames, K, Wm, T, graph, shape):
    """K steps of filter or batch f from a fresh initial cloud, after Wm
    warm-up steps: (GPU ms of the K steps between two events on f's stream,
    wall s, per-kernel times, autotuner result or None, shape the steps ran
    with). With shape=None the autotuner picks the step kernel's workgroup
    shape on the warm filter two steps before the end of the warm-up (so that
    a graph is recorded again before the timed steps); otherwise the given
    shape is set before the warm-up. With graph=True the timed steps replay
    the step's HIP graph, and the per-kernel times come from a second pass
    over the same K steps with plain launches and kernel timing on (the two
    exclude each other)."""
    f.graph(graph)
    tune = shape is None
    if not tune:
        (f.set_shape if hasattr(f, "set_shape") else f.set_shapes)(shape)
    tuned = None
    tune_at = max(Wm - 2, 0)
    for k in range(Wm):
        f.step(frames[k % T])
        if tune and k == tune_at:
            ms, chosen = f.autotune(frames[(k + 1) % T], reps=5)
            tuned = {"ms_per_launch": ms, "chosen": chosen}
    if tune and tuned is None:
        ms, chosen = f.autotune(frames[0], reps=5)
        tuned = {"ms_per_launch": ms, "chosen": chosen}
    ran = tuned["chosen"] if tune else shape
    f.reset()
    torch.cuda.synchronize()
    if not graph:
        f.profile(True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(f.stream)
    for k in range(K):
        f.step(frames[k % T])
    ev1.record(f.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    if graph:
        # the same K steps again from the same initial cloud: they end in the
        # same state, bit for bit, which the caller then reads
        f.graph(False)
        f.reset()
        f.profile(True)
        for k in range(K):
            f.step(frames[k % T])
    kt = f.kernel_times()
    return gpu_ms, wall, kt, tuned, ran


def host_cpu():
    """(CPU model name, logical cores this process may run on)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    return model, cores


def oracle_model(w, n, init_kind):
    """The oracle's model of a single-filter workload with n particles."""
    import oracle
    x0, x1, y0, y1 = w.get("box", (0, w["W"], 0, w["H"]))
    I = w.get("I", 30.0)
    resample, group, _ = w.get("scheme", (0, 256, 0))
    return oracle.Model(n=n, width=w["W"], height=w["H"], s=w["s"], b=10.0, sigma=3.0,
                        patch=w["P"], init_kind=init_kind, init_a=(x0, y0, -1, -1, I / 2),
                        init_b=(x1, y1, 1, 1, 1.5 * I), ess_threshold=w["thr"], seed=1,
                        resample={1: 1, 3: 2}.get(resample, 0), rna_group=group,
                        rna_exchange=w.get("rho", 0.1), arna_min=w.get("rho_min", 0.0))


def cpu_baseline(w, frames, sample_n, sample_t, init_kind, threads):
    """The oracle as it stands on a bounded sample (the first `sample_t`
    frames of the same movie with `sample_n` particles), once on one host
    thread and once on `threads` (its per-particle loops of propagation and
    Eq. 4 in parallel, every reduction sequential: the same results)."""
    import oracle
    model, _ = host_cpu()
    out = {}
    for th, n_s in ((1, sample_n), (threads, sample_n * max(1, min(threads, 16)) // 4)):
        used = oracle.set_threads(th)
        m = oracle_model(w, n_s, init_kind)
        t0 = time.perf_counter()
        r = oracle.run(m, frames[:sample_t], sample_t)
        dt = time.perf_counter() - t0
        if r.status != 0:
            raise SystemExit(f"oracle run failed ({r.status})")
        out[used] = {"value": n_s * sample_t / dt, "unit": "particle updates/s", "cores": used,
                     "kind": "oracle",
                     "sample": f"{sample_t} frames x {n_s} particles of the same workload "
                               f"(fp64, {used} host thread{'s' if used > 1 else ''}, {dt:.1f} s)",
                     "cpu_model": model}
    best = out[max(out)]
    best["single_thread"] = {k: v for k, v in out[1].items() if k != "cpu_model"}
    return best


class GateError(Exception):
    """The filter's output failed a correctness check: no figure is printed."""


def check_state(ppf, f, w, mv, k_truth, scheme):
    """Checks on the GPU's own output after the timed steps, none of which
    uses the oracle: the final ESS (finite, at least 1), the tracking error against the synthetic
    truth (single spot, proportional resampling: at most 1 px), the
    normalised weights summing to one with the reported ESS and estimate,
    and the resampling invariants of the last step (systematic: ancestors
    non-decreasing; systematic and RPA: each particle's offspring count
    within one of N w; RNA: every slot's ancestor in its own group, or in the
    group before for the exchanged tail)."""
    import math

    import numpy as np
    st = f.stats()
    n = f.n
    # 1 / sum w^2 >= 1 for normalised weights; 1 itself is a degenerate cloud,
    # all weight on one particle, which is still a valid state
    if not (math.isfinite(st["ess"]) and st["ess"] >= 1.0 - 1e-9):
        raise GateError(f"final ESS {st['ess']}")
    err = float(np.linalg.norm(st["mean"][:2] - mv.truth[k_truth, 0]))
    if scheme not in (1, 3) and not err <= 1.0:
        raise GateError(f"tracking error {err:.3f} px")
    x, lw, anc = f.particles()
    wt = np.exp(lw)
    tot = math.fsum(wt)
    if not abs(tot - 1.0) < 1e-5:
        raise GateError(f"weights sum to {tot}")
    if not math.isclose(1.0 / float(np.dot(wt, wt)), st["ess"], rel_tol=1e-4):
        raise GateError("ESS does not match the weights")
    mean = np.array([np.dot(wt, x[d].astype(np.float64)) for d in range(5)])
    if not np.abs(mean - st["mean"]).max() <= 1e-3:
        raise GateError(f"estimate {st['mean']} does not match the weights {mean}")
    if st["resampled"]:
        if anc.min() < 0 or anc.max() >= n:
            raise GateError("ancestor out of range")
        if scheme in (1, 3):
            grp = w["scheme"][1]
            g = np.arange(n) // grp
            if scheme == 1:
                moved = int(math.floor(float(np.float32(w.get("rho", 0.1))) * grp))
                src = (g - 1) % (n // grp)
            else:  # ARNA: the tail of each group from one other group (its ring predecessor)
                moved = f.arna_state()["moved"]
                src = (anc // grp).reshape(-1, grp)[:, -1][g] if moved else g
            tail = (np.arange(n) % grp) >= grp - moved
            if not np.array_equal(anc // grp, np.where(tail, src, g)):
                raise GateError("RNA ancestor outside its group or its ring predecessor")
        else:
            if scheme == 0 and np.any(np.diff(anc) < 0):
                raise GateError("systematic ancestors not non-decreasing")
            cnt = np.bincount(anc, minlength=n)
            if np.any(np.abs(cnt - n * wt) >= 2.0) or np.any(cnt[wt == 0] > 0):
                raise GateError("offspring counts off their floor/ceil of N w")
    return err, st


def oracle_check_step(f, w, frames, frames_dev, T, init_kind):
    """One more step after the timed ones, checked against the oracle on
    sampled particles: their propagation from the GPU's parents, their log
    weights (Eq. 4 plus the carried weight, against the GPU's log weight plus
    its normaliser; relative 1e-5 where it matters), and, for systematic
    resampling, every ancestor (the oracle's resampling of the GPU's weights
    with the same uniform: identical outside a 1e-9 band around the CDF
    steps)."""
    import math

    import numpy as np

    import oracle
    n = f.n
    x0, lw0, anc0 = f.particles()
    st0 = f.stats()
    k = st0["k"] + 1
    obs = frames[(k - 1) % T]
    f.step(frames_dev[(k - 1) % T])
    x1, lw1, anc1 = f.particles()
    st1 = f.stats()
    if st1["k"] != k:
        raise GateError("the checked step did not commit")
    rng = np.random.default_rng(k)
    idx = np.unique(np.concatenate([rng.integers(0, n, 4000), [0, 255, 256, 2047, 2048, n - 1],
                                    np.arange(max(0, n - 300), n)]))
    ms = oracle_model(w, idx.size, init_kind)
    par = anc0[idx] if st0["resampled"] else idx
    xo = oracle.propagate_indexed(ms, k, idx, x0[:, par].astype(np.float64))
    tol = np.spacing(np.abs(xo).astype(np.float32)).astype(np.float64) + 1e-6
    if not np.all(np.abs(x1[:, idx] - xo) <= tol):
        raise GateError("propagation differs from the oracle")
    if st0["resampled"]:
        if w.get("scheme", (0,))[0] in (1, 3):
            return  # RNA, ARNA: the carried group weights are checked by the tests
        lw_in = np.full(idx.size, -math.log(n))
    else:
        lw_in = lw0[idx]
    l_orc = lw_in + oracle.loglik(ms, obs, x1[:, idx].astype(np.float64))
    l_gpu = lw1[idx] + st1["delta"]
    rel = np.abs(np.expm1(l_gpu - l_orc))
    if not rel[l_orc - st1["max_logw"] >= -40].max(initial=0.0) <= 1e-5:
        raise GateError("log weights differ from the oracle")
    if st1["resampled"] and w.get("scheme", (0,))[0] == 0:
        wt = np.exp(lw1)
        u = oracle.resample_uniform(ms, k)
        ao = oracle.resample_systematic(wt, u)
        mism = np.nonzero(ao != anc1)[0]
        if mism.size:
            C = np.cumsum(wt)
            us = (mism + u) / n
            j = np.searchsorted(C, us)
            d = np.minimum(np.abs(us - C[np.clip(j - 1, 0, n - 1)]),
                           np.abs(C[np.clip(j, 0, n - 1)] - us))
            if np.any(d > 1e-9):
                raise GateError(f"{int((d > 1e-9).sum())} ancestors differ from the oracle")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    # the card reaches its steady clocks after about 50 ms of load (measured:
    # 1.29 ms per step after 2 warm-up steps, 1.19 ms after 40, and 1.19 ms
    # averaged over 100 steps after 2)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="sir_1024x1024_n38m_p13", choices=sorted(WORKLOADS))
    ap.add_argument("--init", default="uniform", choices=["uniform", "stratified", "uniform-unordered"],
                    help="initial cloud: uniform (the paper's i.i.d. uniform draws, placed in Z "
                         "order), stratified (Z-order strata), uniform-unordered (in draw order)")
    ap.add_argument("--no-alt-init", action="store_true",
                    help="skip the second measurement from the other initial cloud")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--launch", default="stream", choices=["stream", "graph"],
                    help="timed steps as plain launches or as replays of one HIP graph")
    ap.add_argument("--shape", type=int, default=None,
                    help="step-kernel workgroup shape (batched: shape candidate) for every "
                         "step; default: the autotuner picks it during the warm-up")
    ap.add_argument("--no-autotune", action="store_true",
                    help="the same as --shape 0")
    ap.add_argument("--cpu-sample", type=int, default=1 << 22)
    ap.add_argument("--cpu-frames", type=int, default=2)
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="host threads of the all-cores oracle timing (default: the cores this "
                         "process may use, at most OMP_NUM_THREADS when that is set)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_DB", "WRITE_DB"),
                    help="write a traffic record from two counter databases and exit")
    ap.add_argument("--traffic-kernel", default="k_step", choices=sorted(TRAFFIC_GROUPS))
    ap.add_argument("--grad-check", action="store_true",
                    help="the differentiable-SIR experiment (derivatives against central "
                         "differences, gradient ascent) instead of a throughput figure")
    ap.add_argument("--ascent-steps", type=int, default=50)
    args = ap.parse_args()
    if args.no_autotune and args.shape is None:
        args.shape = 0
    if args.traffic_from:
        if args.shape is None:
            raise SystemExit("--traffic-from needs the --shape the counter runs used")
        dbs = []
        for p in args.traffic_from:
            dbs.append(p if p.endswith(".db") else sorted(glob.glob(os.path.join(p, "*.db")))[0])
        rec = traffic_from(dbs[0], dbs[1], args.workload, args.copy_probe_mib or 1024,
                           args.warmup, args.steps, args.shape, args.traffic_kernel)
        print(json.dumps(rec))
        return
    if args.grad_check:
        run_grad_check(args)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    try:
        run(args)
    except GateError as e:
        print(f"bench.py: correctness check failed, no figure reported: {e}", file=sys.stderr)
        sys.exit(3)


def cpu_threads(args):
    if args.cpu_threads > 0:
        return args.cpu_threads
    _, cores = host_cpu()
    env = os.environ.get("OMP_NUM_THREADS", "")
    return min(cores, int(env)) if env.isdigit() and int(env) > 0 else cores


def run(args):
    import numpy as np
    import torch

    import paper_1310_5045_amd as ppf
    from paper_1310_5045_amd import synth

    w = WORKLOADS[args.workload]
    if "tracks" in w:
        return run_multitrack(args, w)
    init_kind = INIT_KINDS[args.init](ppf)
    K, Wm = args.steps, args.warmup
    T = max(K, w["T"])  # the warm-up steps cycle through these frames
    box = w.get("box")
    mv = synth.render_movie(w["W"], w["H"], T, intensity=w.get("I", 30.0), sigma=w["s"],
                            background=10.0, noise_sd=3.0, seed=1,
                            start_box=None if box is None else tuple(float(v) for v in box))
    if w.get("init_radius"):
        # the initial cloud's box around the spot's first position
        x0, y0 = mv.truth[0, 0]
        r = w["init_radius"]
        w = dict(w, box=(x0 - r, x0 + r, y0 - r, y0 + r))
    torch.cuda.set_device(0)
    frames = torch.from_numpy(mv.frames).cuda()
    if args.copy_probe_mib:
        src = torch.ones(args.copy_probe_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    graph = args.launch == "graph"
    plain = None
    if w.get("grad"):
        # the same configuration without derivatives, launched the same way,
        # for the ratio
        pf = ppf.Filter(make_params(ppf, w, init_kind))
        pms, _, pkt, _, _ = timed_steps(torch, pf, frames, K, Wm, T, graph, args.shape)
        pf.close()
        plain = {"value": w["n"] * K / (pms / 1e3), "ms_per_step": pms / K,
                 "k_step_ms": pkt.get("k_step", (1, 0.0))[1] / K}
    f = ppf.Filter(make_params(ppf, w, init_kind, grad=w.get("grad", 0)))
    scheme = w.get("scheme", (0,))[0]
    gpu_ms, wall, kt, tuned, ran = timed_steps(torch, f, frames, K, Wm, T, graph, args.shape)
    err, st = check_state(ppf, f, w, mv, (K - 1) % T, scheme)
    n = w["n"]
    ms_per_step = gpu_ms / K
    value = n * K / (gpu_ms / 1e3)

    P = w["P"]
    step_launches, step_ms = kt.get("k_step", (0, 0.0))
    step_avg_s = step_ms / max(step_launches, 1) / 1e3
    # algorithmic: the separable form's P^2 residual FMAs and P^2
    # square-accumulate FMAs per particle (the count the roofline is taken on)
    flops_per_particle = 4 * P * P
    achieved_tf = flops_per_particle * n / step_avg_s / 1e12
    # executed fp64 flops of the patch sums where the row-sum table serves
    # sum D^2 (converged frames): P (P - 1) row FMAs, P each for the row
    # weights, sum g_y^2, the table adds and two g_y recurrence products
    executed = 2 * P * (P - 1) + 2 * P + 2 * P + P + 2 * P
    # resampling: read 4 B log weight, write 4 B ancestor per particle; the
    # library times the pass (k_anc, then k_fill for queued tile chunks)
    # under one pair of events, per step
    res_launches, res_ms = kt.get("k_resample", (0, 0.0))
    res_avg_s = res_ms / max(res_launches, 1) / 1e3
    res_gbs = 8.0 * n / res_avg_s / 1e9 if res_avg_s > 0 else 0.0
    step_gbs = 48.0 * n / step_avg_s / 1e9

    out = {
        "metric": ("particle updates/s at N=38M on 1 GPU" if n == 38_000_000
                   else f"particle updates/s at N={n} on 1 GPU"),
        "value": value,
        "unit": "particle updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 state, f64 likelihood/normalisation",
        "data": "synthetic",
        "config": {"workload": args.workload, "n_particles": n, "frame": [w["W"], w["H"]],
                   "patch": P, "psf_sigma": w["s"],
                   "resampling": ({0: "systematic", 1: "RNA", 2: "RPA", 3: "ARNA"}[scheme]
                                  + ("" if w["thr"] == float("inf")
                                     else f" when ESS < {w['thr']:.0f}")),
                   "init": args.init, "frames_timed": K, "launch": args.launch,
                   "autotune": tuned, "shape": ran},
        "roofline": {"bound": "alu", "kernel": "k_step", "achieved": achieved_tf,
                     "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved_tf / FP64_VECTOR_PEAK_TFLOPS,
                     "traffic": load_traffic("k_step", args.workload, ran),
                     "avg_launch_ms": step_avg_s * 1e3, "flops_per_particle": flops_per_particle,
                     "flops_basis": "algorithmic: 2 P^2 FMAs of the separable likelihood",
                     "fp64_flops_executed_per_particle": executed,
                     "hbm_gbs_at_48B_per_particle": step_gbs},
        "roofline_resample": {"bound": "hbm", "kernel": "k_anc+k_fill", "achieved": res_gbs,
                              "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": res_gbs / HBM_PEAK_GBS,
                              "traffic": load_traffic("k_resample", args.workload, None),
                              "avg_launch_ms": res_avg_s * 1e3, "bytes_per_particle": 8},
        "kernel_ms_total": {k: v[1] for k, v in kt.items()},
        "kernel_launches": {k: v[0] for k, v in kt.items()},
        "wall_s": wall,
        "tracking_error_px": err,
        "final_ess": st["ess"],
        "checks": "passed",
    }
    if plain is not None:
        g, _ = f.grad()
        out["metric"] = "particle updates/s with d log p^ / d theta (9 parameters) on 1 GPU"
        out["plain_forward"] = plain
        out["ratio_to_plain"] = out["value"] / plain["value"]
        out["grad_cum"] = dict(zip(ppf.GRAD_NAMES, [float(v) for v in g]))
        out["config"]["gradient"] = list(ppf.GRAD_NAMES)
    if not args.no_cpu_baseline and not w.get("grad"):
        # the cpu_baseline leg: one more GPU step checked against the oracle,
        # then the oracle timed on a bounded sample of the workload
        oracle_check_step(f, w, mv.frames, frames, T, init_kind)
        out["checks"] = "passed, with a sampled oracle check of one more step"
    f.close()
    if not args.no_alt_init and not w.get("grad"):
        # the same workload from the other initial cloud (the paper's is
        # uniform; the stratified cloud gives each workgroup a compact
        # first-frame box)
        alt = "stratified" if args.init == "uniform" else "uniform"
        ak = INIT_KINDS[alt](ppf)
        fa = ppf.Filter(make_params(ppf, w, ak))
        a_ms, _, akt, _, _ = timed_steps(torch, fa, frames, K, 2, T, graph, ran)
        a_err, a_st = check_state(ppf, fa, w, mv, (K - 1) % T, scheme)
        fa.close()
        out["init_alternative"] = {"init": alt, "value": n * K / (a_ms / 1e3),
                                   "ms_per_step": a_ms / K,
                                   "kernel_ms_total": {k: v[1] for k, v in akt.items()},
                                   "tracking_error_px": a_err, "final_ess": a_st["ess"]}
    if not args.no_cpu_baseline:
        # (the oracle's run includes its initialisation; the Z-ordered cloud's
        # sort would add to it, and the order does not change the oracle's
        # per-particle work, so it times the same draws unordered)
        ck = ppf.INIT_UNIFORM if init_kind == ppf.INIT_UNIFORM_ZORDER else init_kind
        out["cpu_baseline"] = cpu_baseline(w, mv.frames, min(args.cpu_sample, n), args.cpu_frames,
                                           ck, cpu_threads(args))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
