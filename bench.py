#!/usr/bin/env python3
"""Closest-hit throughput on the 12.6M-tet scene (one MI355X).

Workload: the unit cube as a 128^3 Kuhn grid (12,582,912 tets, 2,146,689
points, interior vertices jittered by +-0.1 cell), constrained faces on the
boundary of a union of 20 seeded spheres; 1920x1080 primary rays from a camera
at (0.5, 0.5, 0.02) looking +z with a 60 degree horizontal field of view
(emitted in 8x8 pixel tiles), then 8 cosine-weighted ambient-occlusion rays
(tmax 0.1) from every primary hit.  The AO ray set is built once, before
timing, from the library's own primary hits.

One step = the camera located once on the device (tetmesh_locate) +
trace_closest on all primary rays, started in that tet + binning of the AO rays
+ trace_closest on the AO rays (each starts from its hit face).  Inputs
are resident in device memory when timing starts; the mesh upload is timed
separately.  Kernel times come from HIP events on the launch stream.

Prints one JSON line (metric, value in Mrays/s, roofline of the dominant
kernel, CPU-oracle baseline).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E peak, GB/s
# VALU issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one operation per lane per
# cycle (an FMA counted once; no packed FP32) = 39.3 T lane-operations/s
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# algorithmic operations of one walk step (the method's arithmetic and bookkeeping,
# counted per ray): fourth vertex id 3 xor; projection of the new point (Eq. 3-5) 8;
# Algorithm 1: two 2-D determinants and two sign tests 8; exit vertex 1; its rank
# among the four ids 5; neighbour read 1; face update 3; termination test 1 = 30.
# Tet16 (Algorithms 6-7) adds the rank of the new vertex 5, one more read and 2 xor;
# Tet32N one more read; Tet32 (Algorithms 2-3) finds the neighbour by 3 compares with
# the stored ids instead of the rank (28).  With tmax: the new point's depth 3, its slot 1, min of the
# face's depths and the test 3.
ALG_OPS_STEP = {"tet20": 30, "tet16": 38, "tet32n": 31, "tet32": 28}
ALG_OPS_TMAX = 7
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_trace_ao_rays_12.6M_tets_hbm_traffic.md")
L1_SUMMARY = os.path.join(ROOT, "profiles", "l1_line_rate_probe.md")
CLOCK_HZ = 2.4e9
N_CUS = 256
# algorithmic bytes of one walk step: the fields the step needs, whatever the layout --
# the xor field (4 B), one neighbour field (4 B) and the new point (12 B)
STEP_BYTES = 20
RAY_IO_BYTES = 24 + 16         # origin + direction in, tri + t + bary out
OPT_INPUT_BYTES = 4            # per optional per-ray input (tmax, start face, start tet)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="paper",
                    choices=["paper", "paper160", "tiny", "batch64", "serve", "ablate", "l1probe", "precision"],
                    help="batch64: 64 uneven meshes in one batched launch; serve: Poisson request "
                         "stream over 16 resident meshes; ablate: record layouts x curve orders and "
                         "camera distances on the 12.6M-tet scene; l1probe: the L1 cache-line access "
                         "rate for 16-byte lane loads; precision: the float64 re-evaluation variant on "
                         "2M stress rays, speed and agreement with the oracle (each prints its own line)")
    ap.add_argument("--serve-seconds", type=float, default=3.0, help="serve: seconds per offered rate")
    ap.add_argument("--serve-loads", default="0.25,0.5,0.75,0.9",
                    help="serve: offered rates as fractions of the measured capacity")
    ap.add_argument("--serve-big", type=int, default=1, help="serve: include the 12.6M-tet mesh")
    ap.add_argument("--serve-burst", type=int, default=512,
                    help="serve: requests in the burst that measures capacity")
    ap.add_argument("--serve-ring", type=int, default=0,
                    help="serve: launches in flight (0 = the library's default, 1)")
    ap.add_argument("--batch-meshes", type=int, default=64, help="batch64: number of meshes")
    ap.add_argument("--tile", type=int, default=8, help="pixel tile edge for ray order (1 = row-major)")
    ap.add_argument("--sfc", default="hilbert", choices=["hilbert", "hilbert_regions", "morton", "none"])
    ap.add_argument("--layout", default="tet16", choices=["tet20", "tet16", "tet32", "tet32n"])
    ap.add_argument("--block", type=int, default=0, help="threads per block (0 = the library's choice)")
    ap.add_argument("--kernel", type=int, default=0,
                    help="0 auto, 1 one lane per ray, 2 persistent lanes, 3 persistent waves on a work queue")
    ap.add_argument("--refill", type=int, default=0, help="persistent refill threshold (0 = default)")
    ap.add_argument("--queue-chunk", type=int, default=0,
                    help="kernel 3: rays a wave takes from the queue at a time (0 = default)")
    ap.add_argument("--ao", type=int, default=8, help="AO rays per primary hit")
    ap.add_argument("--sort", type=int, default=0, help="ray binning: 0 auto, 1 off, 2 on")
    ap.add_argument("--sort-chunk", type=int, default=0, help="log2 rays per binning chunk (0 = default)")
    ap.add_argument("--sort-dirq", type=int, default=0, help="direction bins per axis (0 = default)")
    ap.add_argument("--sort-cells", type=int, default=0,
                    help="log2 origin cells per axis for binning (0 = by direction only)")
    ap.add_argument("--eye", default="", help="camera position x,y,z (default: the workload's)")
    ap.add_argument("--locate", default="shared", choices=["shared", "per-ray"],
                    help="primary rays: camera located once per pass (shared) or by every ray")
    ap.add_argument("--eps", type=float, default=0.0,
                    help="precision variant threshold for both passes (0 = plain float32 walk)")
    ap.add_argument("--passes", type=int, default=0, help="precision variant: 2 = the two-pass form")
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="oracle threads for the CPU baseline (0 = the host's CPUs, at most 16)")
    ap.add_argument("--cpu-stride", type=int, default=1,
                    help="oracle sample: every n-th primary ray and the AO rays of its hits")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run a device copy of this size (counter calibration runs)")
    return ap.parse_args()


def workload(name):
    from synth import config_mesh
    if name in ("paper", "paper160"):
        return config_mesh(name), (0.5, 0.5, 0.02), 1920, 1080
    return config_mesh("tiny"), (0.5, 0.5, 0.05), 64, 64


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the mesh is replicated and rays are independent, so a "
              "multi-GPU run would only shard the ray batch; run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2103_02309_amd.build import LIB, build_library
    if not os.path.exists(LIB):
        build_library(force=True)
    import paper_2103_02309_amd as tetrt
    from synth import pinhole_rays, ao_rays, tri_geometry

    if not torch.cuda.is_available():
        raise RuntimeError("bench.py needs a HIP device")
    dev = torch.device("cuda:0")
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    if args.workload == "batch64":
        return bench_batch(args, tetrt, dev, log)
    if args.workload == "serve":
        return bench_serve(args, tetrt, dev, log)
    if args.workload == "ablate":
        return bench_ablate(args, tetrt, dev, log)
    if args.workload == "l1probe":
        return bench_l1probe(args, tetrt, dev, log)
    if args.workload == "precision":
        return bench_precision(args, tetrt, dev, log)

    t0 = time.time()
    m, eye, W, H = workload(args.workload)
    if args.eye:
        eye = tuple(float(v) for v in args.eye.split(","))
    log("mesh: %d tets, %d points (%.1f s)" % (m.n_tets, m.n_points, time.time() - t0))
    t0 = time.time()
    mesh = tetrt.upload(m.points, m.tets, m.nbrs, m.cflag, sfc=args.sfc, layout=args.layout)
    torch.cuda.synchronize()
    upload_s = time.time() - t0
    info = mesh.info
    log("upload: %.2f s, %d triangles, hot %.1f MB" % (upload_s, info["n_tris"], info["hot_bytes"] / 1e6))

    o, d, pix = pinhole_rays(eye, W, H, 60.0, tile=args.tile)
    po, pd = torch.from_numpy(o).to(dev), torch.from_numpy(d).to(dev)
    n_p = o.shape[0]
    # the pinhole's rays share one origin: it is located once per pass on the device
    # (tetmesh_locate) and broadcast as every primary ray's start tet, as the paper
    # locates the camera once; --locate per-ray has every ray locate it again
    cam = torch.tensor([list(eye)], dtype=torch.float32, device=dev)
    cam_tet = torch.empty(1, dtype=torch.int32, device=dev)
    start_p = torch.empty(n_p, dtype=torch.int32, device=dev) if args.locate == "shared" else None

    def locate_camera():
        if start_p is not None:
            tetrt.tetmesh_locate(mesh.handle, cam, cam_tet)
            start_p.copy_(cam_tet.expand(n_p))
        return start_p

    # set-up pass (untimed): primary hits -> AO rays, step counts for the byte model
    res = mesh.trace(po, pd, start_tet=locate_camera(), want_steps=True)
    torch.cuda.synchronize()
    tri = res["tri"].cpu().numpy()
    tp = res["t"].cpu().numpy()
    steps_p = res["steps"].cpu().numpy().astype(np.int64)
    hit = tri >= 0
    if np.any(tri <= -2):
        raise RuntimeError("primary pass produced %d aborted/invalid rays" % int((tri <= -2).sum()))
    hp = o[hit].astype(np.float64) + tp[hit, None].astype(np.float64) * d[hit].astype(np.float64)
    tv = mesh.tri_vertices(tri[hit])
    nrm, _ = tri_geometry(m.points, tv)
    ao, ad, atm, parent = ao_rays(hp, nrm, d[hit], k=args.ao, seed=3, tmax=0.1)
    sf = tri[hit][parent].astype(np.int32)
    ao_t, ad_t = torch.from_numpy(ao).to(dev), torch.from_numpy(ad).to(dev)
    atm_t, sf_t = torch.from_numpy(atm).to(dev), torch.from_numpy(sf).to(dev)
    n_a = ao.shape[0]
    res_a = mesh.trace(ao_t, ad_t, tmax=atm_t, start_face=sf_t, want_steps=True)
    torch.cuda.synchronize()
    tri_a = res_a["tri"].cpu().numpy()
    steps_a = res_a["steps"].cpu().numpy().astype(np.int64)
    if np.any(tri_a <= -2):
        raise RuntimeError("AO pass produced %d aborted/invalid rays" % int((tri_a <= -2).sum()))
    del res, res_a
    log("rays: %d primary (hit %.3f, mean steps %.1f), %d AO (hit %.3f, mean steps %.1f)" % (
        n_p, hit.mean(), steps_p.mean(), n_a, (tri_a >= 0).mean(), steps_a.mean()))

    # preallocated outputs: no allocation inside the timed loop
    out_p = {"tri": torch.empty(n_p, dtype=torch.int32, device=dev),
             "t": torch.empty(n_p, dtype=torch.float32, device=dev),
             "bary": torch.empty((n_p, 2), dtype=torch.float32, device=dev)}
    out_a = {"tri": torch.empty(n_a, dtype=torch.int32, device=dev),
             "t": torch.empty(n_a, dtype=torch.float32, device=dev),
             "bary": torch.empty((n_a, 2), dtype=torch.float32, device=dev)}

    # binning: the library's automatic rule (batches of at least 2^18 rays that carry
    # tmax), run as its own kernel so that the walk kernel is timed apart
    kw = dict(block=args.block, kernel=args.kernel, refill=args.refill, eps=args.eps, passes=args.passes,
              queue_chunk=args.queue_chunk)
    skw = dict(sort_chunk_log2=args.sort_chunk, sort_dirq=args.sort_dirq, sort_cells_log2=args.sort_cells)
    bin_p = args.sort == 2
    bin_a = args.sort == 2 or (args.sort == 0 and n_a >= (1 << 18))
    ord_p = torch.empty(n_p, dtype=torch.int32, device=dev) if bin_p else None
    ord_a = torch.empty(n_a, dtype=torch.int32, device=dev) if bin_a else None

    def launch(ev=None):
        rec = (lambda k: ev[k].record()) if ev else (lambda k: None)
        rec(0)
        if bin_p:
            mesh.bin_rays(po, pd, ord_p, **skw)
        rec(1)
        mesh.trace_into(out_p, po, pd, start_tet=locate_camera(), order=ord_p, sort=1, **kw)
        rec(2)
        if bin_a:
            mesh.bin_rays(ao_t, ad_t, ord_a, **skw)
        rec(3)
        mesh.trace_into(out_a, ao_t, ad_t, tmax=atm_t, start_face=sf_t, order=ord_a, sort=1, **kw)
        rec(4)

    for _ in range(args.warmup):
        launch()
    if args.copy_probe_mib > 0:
        nbytes = args.copy_probe_mib << 20
        src = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy probe: %d bytes read, %d bytes written" % (nbytes, nbytes))
        del src, dst
    copy_gbs = attainable_copy_gbs(torch, dev)
    torch.cuda.synchronize()

    K = args.steps
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(K)]
    t_wall = time.perf_counter()
    for k in range(K):
        launch(ev[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    seg = lambda a, b: np.array([ev[k][a].elapsed_time(ev[k][b]) for k in range(K)])
    ms_bin_p, ms_p, ms_bin_a, ms_a = seg(0, 1), seg(1, 2), seg(2, 3), seg(3, 4)
    ms_step = float(ev[0][0].elapsed_time(ev[K - 1][4]) / K)
    rays = n_p + n_a
    value = rays / (ms_step * 1e-3) / 1e6

    # algorithmic bytes per launch: per-ray I/O plus 20 B per walk step
    bytes_p = int(steps_p.sum()) * STEP_BYTES + n_p * RAY_IO_BYTES
    bytes_a = int(steps_a.sum()) * STEP_BYTES + n_a * (RAY_IO_BYTES + 2 * OPT_INPUT_BYTES)
    ops_p = int(steps_p.sum()) * ALG_OPS_STEP[args.layout]
    ops_a = int(steps_a.sum()) * (ALG_OPS_STEP[args.layout] + ALG_OPS_TMAX)
    kern = {"primary": (ms_p.mean(), bytes_p, ops_p), "ao": (ms_a.mean(), bytes_a, ops_a)}
    dom = max(kern, key=lambda k: kern[k][0])
    dom_ms, dom_bytes, dom_ops = kern[dom]
    achieved = dom_ops / (dom_ms * 1e-3) / 1e12
    alg_gbs = dom_bytes / (dom_ms * 1e-3) / 1e9
    traffic, l1_acc, l2_req, l2_hit = measured_counters(args) if dom == "ao" else (None,) * 4
    calib = l1_calibration()
    mem = None
    if l1_acc and l2_req and calib:
        cyc = dom_ms * 1e-3 * CLOCK_HZ * N_CUS   # CU-cycles of one launch
        miss = l2_req / l1_acc
        # the calibration's rate at this miss rate, for independent loads and for
        # chained ones (each address from the previous load, as in a walk); the
        # peak is the higher of the two
        ind = l1_peak_at(calib, miss)
        dep_cal = l1_calibration("l1_calibration_dependent")
        dep = l1_peak_at(dep_cal, miss) if dep_cal else None
        peak = max([x for x in (ind, dep) if x], default=None)
        mem = {"l1_lookups_per_cu_cycle": round(l1_acc / cyc, 4), "l1_miss_rate": round(miss, 4),
               "l1_lookup_peak_at_miss_rate": round(peak, 4) if peak else None,
               "l1_frac": round(l1_acc / cyc / peak, 4) if peak else None,
               "l1_lookup_rate_independent_at_miss_rate": round(ind, 4) if ind else None,
               "l1_lookup_rate_dependent_at_miss_rate": round(dep, 4) if dep else None,
               "l2_fills_per_cu_cycle": round(l2_req / cyc, 4)}
    hbm_gbs = traffic / (dom_ms * 1e-3) / 1e9 if traffic else None

    line = {
        "metric": ("closest-hit Mrays/s at 12.6M tets" if args.workload == "paper" else
                   "closest-hit Mrays/s at %.1fM tets" % (m.n_tets / 1e6)),
        "value": round(value, 2),
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": ("kuhn%d-jitter0.1-20spheres, 1920x1080 primary + %d AO/hit (tmax 0.1)" % (
                128 if args.workload == "paper" else 160, args.ao)
                         if args.workload in ("paper", "paper160") else "kuhn16-sphere, 64x64 primary + %d AO/hit" % args.ao),
            "tets": m.n_tets, "points": m.n_points, "triangles": info["n_tris"],
            "primary_rays": n_p, "ao_rays": n_a, "ray_order": "8x8 tiles" if args.tile == 8 else
            ("row-major" if args.tile <= 1 else "%dx%d tiles" % (args.tile, args.tile)),
            "layout": args.layout, "sfc": args.sfc,
            "block": args.block or "auto (128 primary, 256 binned AO)",
            "kernel": {0: "auto", 1: "one lane per ray", 2: "persistent lanes",
                       3: "persistent waves on a per-XCD work queue"}[args.kernel],
            "ray_binning": {0: "auto (AO rays)", 1: "off", 2: "on"}[args.sort], "eye": list(eye),
            "precision_eps": args.eps,
            "primary_start": ("camera located once per pass on the device, shared by every primary ray"
                              if args.locate == "shared" else "every primary ray locates the camera"),
        },
        "roofline": {
            # The dominant kernel (the AO walk) reads far fewer bytes from HBM than
            # the method names (20 B per walk step + ray I/O): its 227 MB hot set sits
            # in the last-level cache and L2 hits 96%.  What binds it is the L1: a
            # wave load whose lanes read distinct lines costs one lookup per line, and
            # the L1 serves lookups at a rate that falls as the share of misses (fills
            # from L2) rises.  So "bound" names the L1, "achieved" is the walk's L1
            # lookups per CU-cycle and "peak" the highest rate the calibration kernel
            # attains at the same miss rate; HBM is reported from measured bytes ("hbm",
            # "traffic"), the method's algorithmic byte rate apart ("algorithmic"),
            # never as an HBM fraction.
            "bound": "l1" if mem and mem["l1_frac"] else None,
            "achieved": mem["l1_lookups_per_cu_cycle"] if mem and mem["l1_frac"] else None,
            "peak": mem["l1_lookup_peak_at_miss_rate"] if mem else None,
            "unit": "L1 lookups per CU per cycle",
            "frac": mem["l1_frac"] if mem else None,
            "traffic": traffic,
            "kernel": "k_trace (%s rays)" % dom, "kernel_ms": round(float(dom_ms), 4),
            "hbm": {"achieved": round(hbm_gbs, 1) if hbm_gbs else None, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(hbm_gbs / HBM_PEAK_GBS, 4) if hbm_gbs else None,
                    "measured_bytes_per_launch": traffic, "copy_attainable_gbs": copy_gbs,
                    "l2_hit_rate": l2_hit},
            "algorithmic": {"bytes_per_launch": dom_bytes, "gbs": round(alg_gbs, 1),
                            "gbs_over_hbm_peak": round(alg_gbs / HBM_PEAK_GBS, 4),
                            "note": "20 B per walk step + ray I/O per launch / kernel time; "
                                    "served mostly from L2 and the last-level cache"},
            "alu": {"achieved": round(achieved, 2), "peak": round(ALU_PEAK_TOPS, 2), "unit": "TOP/s",
                    "frac": round(achieved / ALU_PEAK_TOPS, 4), "algorithmic_ops": dom_ops},
            "memory_pipeline": mem,
            "primary_walk": {"bound": "alu (VALU issue)", "kernel_ms": round(float(ms_p.mean()), 4),
                             "alu_frac": round(ops_p / (ms_p.mean() * 1e-3) / 1e12 / ALU_PEAK_TOPS, 4),
                             "algorithmic_gbs": round(bytes_p / (ms_p.mean() * 1e-3) / 1e9, 1)},
        },
        "detail": {
            "primary_ms": round(float(ms_p.mean()), 4), "ao_ms": round(float(ms_a.mean()), 4),
            "primary_binning_ms": round(float(ms_bin_p.mean()), 4) if bin_p else None,
            "ao_binning_ms": round(float(ms_bin_a.mean()), 4) if bin_a else None,
            "primary_mrays_s": round(n_p / ms_p.mean() / 1e3, 2),
            "ao_mrays_s": round(n_a / ms_a.mean() / 1e3, 2),
            "primary_mean_steps": round(float(steps_p.mean()), 2),
            "ao_mean_steps": round(float(steps_a.mean()), 2),
            "primary_hit_rate": round(float(hit.mean()), 4),
            "ao_hit_rate": round(float((tri_a >= 0).mean()), 4),
            "primary_alg_gbs": round(bytes_p / (ms_p.mean() * 1e-3) / 1e9, 1),
            "ao_alg_gbs": round(bytes_a / (ms_a.mean() * 1e-3) / 1e9, 1),
            "upload_s": round(upload_s, 2), "host_wall_s": round(wall, 3),
            "hot_bytes": info["hot_bytes"],
        },
        "cpu_baseline": None,
    }

    if args.cpu_baseline:
        threads = args.cpu_threads or min(16, len(os.sched_getaffinity(0)))
        line["cpu_baseline"] = cpu_baseline(m, o, d, ao, ad, atm, sf, parent, hit, args.cpu_stride,
                                            threads, log)
    mesh.free()
    print(json.dumps(line), flush=True)


def kernel_source_hash():
    """sha256 of the walk kernel's sources, to tell whether a counter summary
    still describes the kernel that runs."""
    import hashlib
    h = hashlib.sha256()
    for f in ("walk.hip", "device.h"):
        with open(os.path.join(ROOT, "paper_2103_02309_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def summary_values(path, keys):
    """`key = value` lines of a committed counter summary."""
    try:
        text = open(path).read()
    except OSError:
        return {}
    vals = {}
    for line in text.splitlines():
        line = line.strip().strip("`")
        if "=" in line and line.startswith(keys):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip().strip("`")
    return vals


def measured_counters(args):
    """HBM bytes, L1 lookups and L1 fills from L2 per launch of the AO walk, from
    the committed rocprofv3 counter summary (HBM: FETCH_SIZE x 2.0 + WRITE_SIZE x
    1.0, scaled by a device copy; TCP_TOTAL_CACHE_ACCESSES; TCP_TCC_READ_REQ), or
    None for each when the summary was taken on other kernel sources or another
    setup."""
    keys = ("traffic_bytes_per_launch", "l1_accesses_per_launch", "l2_requests_per_launch", "l2_hit_rate")
    if (args.layout != "tet16" or args.sfc != "hilbert" or args.sort != 0 or args.block not in (0, 256) or args.eps > 0
            or args.kernel not in (0, 1)):
        return (None,) * len(keys)
    vals = summary_values(TRAFFIC_SUMMARY, keys + ("kernel_source_sha256",))
    if vals.get("kernel_source_sha256") != kernel_source_hash():
        return (None,) * len(keys)
    out = []
    for k in keys:
        try:
            out.append(float(vals[k]) if k == "l2_hit_rate" else int(vals[k]))
        except (KeyError, ValueError):
            out.append(None)
    return tuple(out)


def attainable_copy_gbs(torch, dev, nbytes=1 << 30, reps=5):
    """Device-to-device copy bandwidth on this GPU (bytes read + written per
    second, median of `reps` 1 GiB copies): the HBM rate a streaming kernel
    attains, beside the 8 TB/s peak."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    ms = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        ms.append(a.elapsed_time(b))
    del src, dst
    return round(2 * nbytes / (sorted(ms)[reps // 2] * 1e-3) / 1e9, 1)


def l1_calibration(key="l1_calibration"):
    """The calibration kernel's L1 lookup rate for random 16-byte lane loads
    against its L1 miss rate, [(miss_rate, lookups per CU-cycle)] sorted by miss
    rate, from the committed summary; None if absent.  ``l1_calibration``:
    independent loads (the L1's throughput); ``l1_calibration_dependent``: each
    lane's loads a chain, each address depending on the previous load."""
    vals = summary_values(L1_SUMMARY, (key,))
    try:
        pts = sorted((float(a), float(b)) for a, b in (x.split(":") for x in vals[key].split(",")))
    except (KeyError, ValueError):
        return None
    return pts if len(pts) >= 2 else None


def l1_peak_at(calib, miss):
    """Lookup rate the calibration reaches at L1 miss rate ``miss``: cycles per
    lookup interpolated linearly between the two calibrated miss rates around it
    (None outside their range)."""
    for (m0, r0), (m1, r1) in zip(calib, calib[1:]):
        if m0 <= miss <= m1:
            w = (miss - m0) / (m1 - m0) if m1 > m0 else 0.0
            return 1.0 / ((1.0 - w) / r0 + w / r1)
    return None


def bench_precision(args, tetrt, dev, log):
    """The precision variant on the stress set: 2,000,000 rays on the 16^3 scene
    (10% aimed through mesh vertices, 10% along non-surface edges, 80% random),
    for eps = 0 (plain float32 walk) and the sweep 1e-7 .. 1e-4: walk time and
    Mrays/s (every ray locates its own origin), step caps, invalid results and
    the share of steps decided in float64.  Its CPU-baseline leg (on unless
    --cpu-baseline 0) runs the FP64 oracle on the same rays, reports its rate, and
    per ray kind the share of rays whose triangle differs from the oracle's, how
    many of those are not explained by an edge/vertex tie, and the largest t and
    barycentric errors of the matched hits."""
    import numpy as np
    import torch
    from synth import config_mesh, precision_rays
    m = config_mesh("tiny")
    n = 2_000_000
    o, d, kind = precision_rays(m.points, m.tets, m.cflag, n=n, seed=4)
    kinds = {0: "random", 1: "through vertices", 2: "along edges"}
    mesh = tetrt.upload(m.points, m.tets, m.nbrs, m.cflag, layout=args.layout)
    O, D = torch.from_numpy(o).to(dev), torch.from_numpy(d).to(dev)
    out = tetrt.outputs(n, dev, want_steps=True)
    out["fp64_steps"] = torch.empty(n, dtype=torch.int32, device=dev)
    rows, results = [], {}
    for eps in (0.0, 1e-7, 1e-6, 1e-5, 1e-4):
        kw = dict(eps=eps, max_steps=20000)
        mesh.trace_into(out, O, D, **kw)   # warm-up, and the results reported below
        torch.cuda.synchronize()
        got = {k: v.cpu().numpy() for k, v in out.items()}
        results[eps] = got
        ms = []
        for _ in range(max(3, args.steps // 4)):
            a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            mesh.trace_into(out, O, D, **kw)
            e.record()
            e.synchronize()
            ms.append(a.elapsed_time(e))
        t = sorted(ms)[len(ms) // 2]
        row = {"eps": eps, "ms": round(t, 4), "mrays_s": round(n / t / 1e3, 1),
               "fp64_step_share": round(float(got["fp64_steps"].sum()) / max(1.0, float(got["steps"].clip(0).sum())), 6)}
        for k, name in kinds.items():
            sel = kind == k
            row[name] = {"rays": int(sel.sum()), "step_caps": int((got["tri"][sel] == -2).sum()),
                         "invalid": int((got["tri"][sel] == -3).sum())}
        rows.append(row)
        log(json.dumps(row))
    mesh.free()
    base = None
    if args.cpu_baseline:
        base = precision_cpu_baseline(args, m, o, d, kind, kinds, results, rows, log)
    print(json.dumps({"metric": "precision variant on 2M stress rays (16^3 scene)", "unit": "Mrays/s",
                      "dtype": "f32 walk, f64 re-evaluation", "data": "synthetic", "rows": rows,
                      "config": {"workload": "kuhn16-sphere, 2M rays: 10% through vertices, 10% along "
                                             "non-surface edges, 80% random", "layout": args.layout},
                      "cpu_baseline": base}), flush=True)


def precision_cpu_baseline(args, m, o, d, kind, kinds, results, rows, log):
    """The precision workload's CPU-baseline leg: the FP64 oracle on all its rays
    (threads over contiguous ranges), its rate, and the GPU results of every eps
    compared with it (the parity rule of oracle/compare.py), added to ``rows``."""
    import numpy as np
    import oracle
    from oracle.compare import compare
    from concurrent.futures import ThreadPoolExecutor
    om = oracle.OracleMesh.from_kuhn(m)
    n = o.shape[0]
    threads = args.cpu_threads or min(16, len(os.sched_getaffinity(0)))
    b = np.linspace(0, n, threads + 1).astype(np.int64)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        parts = list(ex.map(lambda k: om.trace(o[b[k]:b[k + 1]], d[b[k]:b[k + 1]]), range(threads)))
    wall = time.perf_counter() - t0
    ref = {key: np.concatenate([p[key] for p in parts]) for key in parts[0]}
    log("oracle: %d rays in %.1f s on %d threads" % (n, wall, threads))
    for row in rows:
        got = results[row["eps"]]
        ident = 0
        for k, name in kinds.items():
            sel = kind == k
            rep = compare(m.points, om.tri_verts, o[sel], d[sel], {x: v[sel] for x, v in ref.items()},
                          {x: v[sel] for x, v in got.items()})
            ident += rep["identical"]
            row[name].update({"mismatch_rate": round(1.0 - rep["frac_identical"], 7),
                              "unexplained": int(rep["n_unexplained"]),
                              "max_t_rel": float("%.3g" % rep["max_t_rel"]),
                              "max_bary": float("%.3g" % rep["max_bary"])})
        row["identical_all"] = round(ident / n, 6)
    return {"value": round(n / wall / 1e6, 4), "unit": "Mrays/s", "cores": threads, "kind": "oracle",
            "sample": "all %d rays, %.1f s wall on %d threads" % (n, wall, threads)}


_PROBE_MODES = {"random": 0, "8_lanes": 1, "one_line": 2, "chain": 3}
_probe = None


def probe_lib():
    """The benchmark's L1 calibration kernel, libtetrt_probe.so (a library of its
    own, not part of the traversal library), built if absent."""
    global _probe
    if _probe is None:
        import ctypes as C
        from paper_2103_02309_amd.build import PROBE_LIB, build_probe
        if not os.path.exists(PROBE_LIB):
            build_probe(force=True)
        L = C.CDLL(PROBE_LIB)
        vp, i32 = C.c_void_p, C.c_int32
        L.tetrt_probe_l1.argtypes = [vp, C.c_uint64, i32, C.c_uint32, C.c_uint32, i32, i32, vp, vp]
        L.tetrt_probe_l1.restype = i32
        L.tetrt_probe_last_error.argtypes = []
        L.tetrt_probe_last_error.restype = C.c_char_p
        _probe = L
    return _probe


def probe_l1(buf, mode, unit_bytes, units, blocks, iters, out, stream=None):
    """Enqueue the L1 calibration kernel (buf: device bytes, out: a device tensor of
    blocks * 256 * 16 bytes) on stream (default: torch's current one); the caller
    times it."""
    import torch
    if not buf.is_cuda or not out.is_cuda or out.numel() * out.element_size() < blocks * 256 * 16:
        raise ValueError("probe_l1: device buffers, out of at least blocks * 4096 bytes")
    st = stream if stream is not None else torch.cuda.current_stream()
    L = probe_lib()
    rc = L.tetrt_probe_l1(buf.data_ptr(), buf.numel() * buf.element_size(), _PROBE_MODES[mode],
                          int(unit_bytes), int(units), int(blocks), int(iters), out.data_ptr(),
                          st.cuda_stream)
    if rc != 0:
        raise RuntimeError("tetrt_probe_l1 %d: %s" % (rc, L.tetrt_probe_last_error().decode()))


def bench_l1probe(args, tetrt, dev, log):
    """The L1's line-lookup rate for wave loads of 16 bytes per lane, by address
    spread: random 128-byte lines (each lane its own line) in L1-resident,
    L2-resident and HBM-sized sets, and 8 lanes or a whole wave per line."""
    import torch
    blocks, iters = 2048, 2048   # 8 waves per SIMD on 256 CUs, 2048 loads per lane
    buf = torch.ones(128 << 20, dtype=torch.uint8, device=dev)
    out = torch.empty(blocks * 256 * 4, dtype=torch.int32, device=dev)
    cases = [("random", 128, 128, "random 128-B lines, 16 KiB set"),
             ("random", 1 << 14, 128, "random 128-B lines, 2 MiB set"),
             ("random", 1 << 20, 128, "random 128-B lines, 128 MiB set"),
             ("random", 256, 64, "random 64-B units, 16 KiB set"),
             ("random", 1 << 10, 16, "random 16-B units, 16 KiB set"),
             ("random", 1 << 11, 16, "random 16-B units, 32 KiB set"),
             ("random", 1 << 9, 80, "random 16-B reads in 80-B units, 40 KiB set"),
             ("random", 1 << 10, 48, "random 16-B reads in 48-B units, 48 KiB set"),
             ("random", 1 << 12, 16, "random 16-B units, 64 KiB set"),
             ("random", 1 << 14, 16, "random 16-B units, 256 KiB set"),
             ("random", 1 << 17, 16, "random 16-B units, 2 MiB set"),
             ("chain", 1 << 10, 16, "dependent random 16-B units, 16 KiB set"),
             ("chain", 1 << 11, 16, "dependent random 16-B units, 32 KiB set"),
             ("chain", 1 << 9, 80, "dependent random 16-B reads in 80-B units, 40 KiB set"),
             ("chain", 1 << 10, 48, "dependent random 16-B reads in 48-B units, 48 KiB set"),
             ("chain", 1 << 12, 16, "dependent random 16-B units, 64 KiB set"),
             ("chain", 1 << 14, 16, "dependent random 16-B units, 256 KiB set"),
             ("8_lanes", 128, 128, "8 lanes per 128-B line, 16 KiB set"),
             ("one_line", 128, 128, "one 128-B line per wave load, 16 KiB set")]
    st = torch.cuda.current_stream()
    rows = []
    for mode, units, ub, what in cases:
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ms = []
        for rep in range(args.warmup + args.steps):
            a.record(st)
            probe_l1(buf, mode, ub, units, blocks, iters, out, st)
            b.record(st)
            b.synchronize()
            if rep >= args.warmup:
                ms.append(a.elapsed_time(b))
        t = sorted(ms)[len(ms) // 2]
        wave_loads = blocks * 4 * iters
        cycles = t * 1e-3 * CLOCK_HZ
        lines_per_load = {"random": units * (1 - (1 - 1 / units) ** 64) if ub == 128 else None,
                          "chain": None, "8_lanes": 8, "one_line": 1}[mode]
        row = {"case": what, "ms": round(t, 4),
               "lane_loads_per_cu_cycle": round(wave_loads * 64 / N_CUS / cycles, 3),
               "wave_loads_per_cu_cycle": round(wave_loads / N_CUS / cycles, 4)}
        if lines_per_load:
            row["expected_lines_per_wave_load"] = round(lines_per_load, 2)
            row["lines_per_cu_cycle"] = round(wave_loads * lines_per_load / N_CUS / cycles, 3)
        rows.append(row)
        log(json.dumps(row))
    print(json.dumps({"metric": "L1 cache-line lookups per CU per cycle, 16-byte lane loads",
                      "cases": rows, "config": {"blocks": blocks, "block": 256, "iters": iters,
                                                "clock_ghz": CLOCK_HZ / 1e9, "cus": N_CUS}}), flush=True)


def bench_batch(args, tetrt, dev, log):
    """Many-mesh workload: ``--batch-meshes`` Kuhn meshes, n log-uniform in [8, 96],
    1..10 spheres each, 1K..1M rays each (half primary from an interior camera,
    half AO from their hits).  Times the meshes traced one launch each, one
    batched launch, the batched launch as a HIP graph, and the autotuned batch."""
    import numpy as np
    import torch
    from synth.batch import batch_specs, spec_mesh, camera_rays, ao_from_hits

    specs = batch_specs(count=args.batch_meshes, seed=10)
    meshes, jobs, total_tets = [], [], 0
    t0 = time.time()
    for k, spec in enumerate(specs):
        m = spec_mesh(spec)
        mesh = tetrt.upload(m.points, m.tets, m.nbrs, m.cflag, layout=args.layout, sfc=args.sfc)
        total_tets += m.n_tets
        po, pd = camera_rays(spec)
        res = mesh.trace(torch.from_numpy(po).to(dev), torch.from_numpy(pd).to(dev))
        tri = res["tri"].cpu().numpy()
        tp = res["t"].cpu().numpy()
        ao, ad, atm, sf = ao_from_hits(m.points, mesh.tri_vertices, po, pd, tri, tp,
                                       spec["rays"] - len(po), spec["ao_seed"])
        o = np.concatenate([po, ao])
        d = np.concatenate([pd, ad])
        tmax = np.concatenate([np.full(len(po), np.inf, np.float32), atm])
        sfc = np.concatenate([np.full(len(po), -1, np.int32), sf])
        n = len(o)
        jobs.append(dict(mesh=mesh, orig=torch.from_numpy(o).to(dev), dirs=torch.from_numpy(d).to(dev),
                         tmax=torch.from_numpy(tmax).to(dev), start_face=torch.from_numpy(sfc).to(dev),
                         out=tetrt.outputs(n, dev)))
        meshes.append(mesh)
        log("mesh %d/%d: n=%d, %d tets, %d rays (%d AO)  [%.0f s]" % (
            k + 1, len(specs), spec["n"], m.n_tets, n, len(ao), time.time() - t0))
        del m
    rays = sum(int(j["orig"].shape[0]) for j in jobs)
    kw = dict(block=args.block, sort=args.sort, sort_chunk_log2=args.sort_chunk,
              sort_dirq=args.sort_dirq, sort_cells_log2=args.sort_cells, eps=args.eps)
    sep_out = [tetrt.outputs(int(j["orig"].shape[0]), dev) for j in jobs]

    def separate():
        for j, out in zip(jobs, sep_out):
            j["mesh"].trace_into(out, j["orig"], j["dirs"], tmax=j["tmax"], start_face=j["start_face"], **kw)

    def timed(fn, reps):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    b = tetrt.Batch(max_jobs=len(jobs), max_rays=rays)
    b.set(jobs, **kw)
    K = args.steps
    ms_sep = timed(separate, K)
    ms_batch = timed(b.launch, K)
    ms_graph = timed(b.graph_launch, K)
    # persistent waves draining one queue over all jobs, with its defaults (float32
    # walk only)
    ms_queue = ms_queue_graph = None
    if args.eps == 0.0:
        b.set(jobs, kernel=3)
        ms_queue = timed(b.launch, K)
        ms_queue_graph = timed(b.graph_launch, K)
    b.set(jobs, **kw)
    chosen, _ = b.tune(reps=3)
    ms_tuned = timed(b.launch, K)
    ms_tuned_graph = timed(b.graph_launch, K)
    torch.cuda.synchronize()
    # the batched results are those of the separate launches, bit for bit
    mism = 0
    for j, out in zip(jobs, sep_out):
        for key in ("tri", "t", "bary"):
            x, y = j["out"][key], out[key]
            mism += int((~((x == y) | (torch.isnan(x) & torch.isnan(y)))).sum().item())
    best = min(x for x in (ms_batch, ms_graph, ms_queue, ms_queue_graph, ms_tuned, ms_tuned_graph)
               if x is not None)
    r4 = lambda x: None if x is None else round(x, 4)
    line = {
        "metric": "batched closest-hit Mrays/s over %d meshes" % len(jobs),
        "value": round(rays / (best * 1e-3) / 1e6, 2),
        "unit": "Mrays/s", "n_gpus": 1, "steps": K, "warmup": args.warmup,
        "ms_per_step": round(best, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "%d Kuhn meshes n log-uniform 8..96, 1-10 spheres, 1K-1M rays each "
                               "(half primary, half AO)" % len(jobs),
                   "tets": total_tets, "rays": rays, "layout": args.layout, "precision_eps": args.eps,
                   "tuned": chosen},
        "detail": {"separate_launches_ms": round(ms_sep, 4), "batch_ms": round(ms_batch, 4),
                   "batch_graph_ms": round(ms_graph, 4), "queue_ms": r4(ms_queue),
                   "queue_graph_ms": r4(ms_queue_graph), "tuned_ms": round(ms_tuned, 4),
                   "tuned_graph_ms": round(ms_tuned_graph, 4),
                   "separate_mrays_s": round(rays / (ms_sep * 1e-3) / 1e6, 2),
                   "batch_vs_separate": round(ms_sep / best, 3),
                   "mismatches_vs_separate": mism},
    }
    b.free()
    for mesh in meshes:
        mesh.free()
    print(json.dumps(line), flush=True)
    if mism:
        raise SystemExit("batched results differ from separate launches in %d values" % mism)


def bench_serve(args, tetrt, dev, log):
    """Serving: 16 resident meshes (15 of the many-mesh sizes, plus the 12.6M-tet
    scene with --serve-big 1); requests with a uniform interior camera, resolution
    uniform over {64, 256, 512, 1024}^2 and kind primary/shadow/AO at 50/25/25%.
    First the capacity (a burst of requests drained at once), then a Poisson
    stream at each offered fraction of it: p50/p99 latency from arrival to the
    step that sees the request's last launch complete, and the achieved Mrays/s."""
    import numpy as np
    import torch
    from synth import config_mesh
    from synth.batch import batch_specs, spec_mesh

    t0 = time.time()
    hosts = [spec_mesh(s) for s in batch_specs(count=15 if args.serve_big else 16, seed=50)]
    if args.serve_big:
        hosts.append(config_mesh("paper"))
    meshes = []
    for m in hosts:
        meshes.append(tetrt.upload(m.points, m.tets, m.nbrs, m.cflag, layout=args.layout, sfc=args.sfc))
    tets = sum(m.n_tets for m in hosts)
    del hosts
    log("serve: %d meshes, %d tets, uploaded in %.0f s" % (len(meshes), tets, time.time() - t0))
    rng = np.random.default_rng(77)
    sizes = [64, 256, 512, 1024]
    kinds = ["primary", "primary", "shadow", "ao"]

    def request():
        f = rng.normal(size=3)
        f /= np.linalg.norm(f)
        up = (0.0, 1.0, 0.0) if abs(f[1]) < 0.9 else (1.0, 0.0, 0.0)
        S = sizes[int(rng.integers(0, 4))]
        return dict(mesh=int(rng.integers(0, len(meshes))), kind=kinds[int(rng.integers(0, 4))],
                    width=S, height=S, eye=rng.uniform(0.05, 0.95, 3), forward=f, up=up,
                    fov_h_deg=60.0, light=rng.uniform(0.05, 0.95, 3), ao_tmax=0.1,
                    seed=int(rng.integers(0, 1 << 31)))

    # output slots for requests in flight: enough that an arrival never waits for a
    # free one at the offered loads measured (views into three arenas)
    n_buf = 768
    slot = 1024 * 1024
    arena = tetrt.outputs(n_buf * slot, dev)
    bufs = [{k: v[i * slot:(i + 1) * slot] for k, v in arena.items()} for i in range(n_buf)]

    srv = tetrt.Server(meshes, max_rays=32 << 20, block=args.block, sort=args.sort, ring=args.serve_ring)

    # capacity: a burst of requests, drained (long enough that its mix of sizes
    # is close to the stream's)
    # requests are packed before they are submitted (Server.prepare), so the
    # submitting loop costs a few microseconds per request
    burst = [srv.prepare(**request()) for _ in range(args.serve_burst)]
    for _ in range(2):
        for k, r in enumerate(burst):
            srv.submit_prepared(r, bufs[k % n_buf])
            if k % n_buf == n_buf - 1:
                srv.drain()
        srv.drain()
        srv.poll(4096)
    torch.cuda.synchronize()
    t_b = time.perf_counter()
    for k, r in enumerate(burst):
        srv.submit_prepared(r, bufs[k % n_buf])
        if k % n_buf == n_buf - 1:
            srv.drain()
    srv.drain()
    torch.cuda.synchronize()
    burst_s = time.perf_counter() - t_b
    done = srv.poll(4096)
    burst_rays = sum(d["rays"] for d in done)
    cap_rps = len(burst) / burst_s
    log("serve: capacity %.0f requests/s, %.1f Mrays/s (burst of %d)" % (cap_rps, burst_rays / burst_s / 1e6, len(burst)))
    plain = serve_plain_forms(args, tetrt, dev, log, meshes, burst)

    loads = []
    for frac in [float(x) for x in args.serve_loads.split(",") if x]:
        rate = frac * cap_rps
        n_req = max(20, int(rate * args.serve_seconds))
        gaps = rng.exponential(1.0 / rate, n_req)
        reqs = [srv.prepare(**request()) for _ in range(n_req)]
        free = list(range(n_buf))
        owner, arrival, lat, waits = {}, {}, [], []
        rays = 0
        start = time.monotonic_ns()
        due = start + np.cumsum(gaps * 1e9).astype(np.int64)
        nxt = 0
        no_slot = 0
        while len(lat) < n_req:
            now = time.monotonic_ns()
            while nxt < n_req and due[nxt] <= now:
                if not free:
                    no_slot += 1       # the harness has no output slot: counted, never hidden
                    break
                b = free.pop()
                i = srv.submit_prepared(reqs[nxt], bufs[b])
                owner[i] = b
                arrival[i] = int(due[nxt])
                waits.append((now - due[nxt]) * 1e-6)
                nxt += 1
            srv.step()
            for d in srv.poll(4096):
                lat.append((d["done_ns"] - arrival[d["id"]]) * 1e-6)
                rays += d["rays"]
                free.append(owner.pop(d["id"]))
        wall = (time.monotonic_ns() - start) * 1e-9
        lat = np.array(lat)
        waits = np.array(waits)
        # latency counts from the arrival time; the submit loop's own delay (an
        # arrival seen only after the previous step returned) is part of it and is
        # also reported alone
        entry = {"offered_frac": frac, "offered_rps": round(rate, 1), "requests": n_req,
                 "p50_ms": round(float(np.percentile(lat, 50)), 3),
                 "p99_ms": round(float(np.percentile(lat, 99)), 3),
                 "mrays_s": round(rays / wall / 1e6, 2),
                 "submit_delay_p50_ms": round(float(np.percentile(waits, 50)), 3),
                 "submit_delay_p99_ms": round(float(np.percentile(waits, 99)), 3),
                 "waits_for_output_slot": no_slot}
        log("serve: %s" % json.dumps(entry))
        loads.append(entry)
    srv.free()
    for m in meshes:
        m.free()
    line = {
        "metric": "serving p50/p99 latency over 16 resident meshes",
        "value": loads[-1]["p99_ms"] if loads else None, "unit": "ms (p99 at the highest offered load)",
        "n_gpus": 1, "higher_is_better": False, "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "16 meshes (%d tets), Poisson requests: interior camera, "
                               "64^2..1024^2, primary/shadow/AO 50/25/25%%" % tets,
                   "layout": args.layout, "seconds_per_load": args.serve_seconds,
                   "capacity_burst": args.serve_burst, "ring": args.serve_ring or 1},
        "capacity": {"requests_s": round(cap_rps, 1), "mrays_s": round(burst_rays / burst_s / 1e6, 2)},
        "same_burst_plain": plain,
        "served_vs_plain": round(burst_rays / burst_s / 1e6 / plain["plain_mrays_s"], 3),
        "served_vs_batch": round(burst_rays / burst_s / 1e6 / plain["batch_mrays_s"], 3),
        "loads": loads,
    }
    print(json.dumps(line), flush=True)


def serve_plain_forms(args, tetrt, dev, log, meshes, burst):
    """The capacity burst's requests traced without the server: their rays made
    once with tm_request_rays (camera rays, then each secondary ray from its
    camera ray's hit) and resident before timing; then (a) one trace_closest per
    request and phase, (b) one batched launch per phase over every request.
    Walk time only (HIP events); the server's figure also covers ray generation,
    admission and its table copies."""
    import torch
    B = tetrt.binding
    reqs = []
    for r in burst:
        n = r.width * r.height
        d = {"mesh": meshes[r.mesh], "n": n, "kind": r.kind}
        reqs.append(d)
    total = sum(q["n"] for q in reqs)
    sec = [q for q in reqs if q["kind"] != 0]
    log("serve: plain forms over %d requests, %d + %d rays" % (len(reqs), total, sum(q["n"] for q in sec)))
    for q, r in zip(reqs, burst):
        n = q["n"]
        q["p0"] = dict(orig=torch.empty((n, 3), dtype=torch.float32, device=dev),
                       dirs=torch.empty((n, 3), dtype=torch.float32, device=dev),
                       tmax=torch.empty(n, dtype=torch.float32, device=dev),
                       sf=torch.empty(n, dtype=torch.int32, device=dev), out=tetrt.outputs(n, dev))
        p0 = q["p0"]
        B._check(B._load().tm_request_rays(B.C.c_void_p(q["mesh"].handle), B.C.byref(r), 0,
                                           p0["orig"].data_ptr(), p0["dirs"].data_ptr(), p0["tmax"].data_ptr(),
                                           p0["sf"].data_ptr(), None, None, B._stream(None)))
        q["mesh"].trace_into(p0["out"], p0["orig"], p0["dirs"], tmax=p0["tmax"], start_face=p0["sf"])
        if q["kind"] != 0:
            q["p1"] = dict(orig=p0["orig"].clone(), dirs=p0["dirs"].clone(),
                           tmax=torch.empty(n, dtype=torch.float32, device=dev),
                           sf=torch.empty(n, dtype=torch.int32, device=dev), out=tetrt.outputs(n, dev))
            p1 = q["p1"]
            B._check(B._load().tm_request_rays(
                B.C.c_void_p(q["mesh"].handle), B.C.byref(r), 1, p1["orig"].data_ptr(), p1["dirs"].data_ptr(),
                p1["tmax"].data_ptr(), p1["sf"].data_ptr(), p0["out"]["tri"].data_ptr(),
                p0["out"]["t"].data_ptr(), B._stream(None)))
    torch.cuda.synchronize()
    phases = [[q["p0"] for q in reqs], [q["p1"] for q in sec]]
    rays = sum(int(p["orig"].shape[0]) for ph in phases for p in ph)
    kw = dict(block=args.block, sort=args.sort)

    def plain():
        for ph in phases:
            for q, p in zip(reqs if ph is phases[0] else sec, ph):
                q["mesh"].trace_into(p["out"], p["orig"], p["dirs"], tmax=p["tmax"], start_face=p["sf"], **kw)

    batches = []
    for ph, qs in ((phases[0], reqs), (phases[1], sec)):
        b = tetrt.Batch(max_jobs=len(ph), max_rays=sum(int(p["orig"].shape[0]) for p in ph))
        b.set([dict(mesh=q["mesh"], orig=p["orig"], dirs=p["dirs"], tmax=p["tmax"], start_face=p["sf"],
                    out=p["out"]) for q, p in zip(qs, ph)], **kw)
        batches.append(b)

    def batched():
        for b in batches:
            b.launch()

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ms_plain, ms_batch = timed(plain), timed(batched)
    for b in batches:
        b.free()
    res = {"rays": rays, "plain_ms": round(ms_plain, 3), "plain_mrays_s": round(rays / ms_plain / 1e3, 1),
           "batch_ms": round(ms_batch, 3), "batch_mrays_s": round(rays / ms_batch / 1e3, 1),
           "launches_plain": len(phases[0]) + len(phases[1]), "launches_batch": 2}
    log("serve: plain forms %s" % json.dumps(res))
    return res


def bench_ablate(args, tetrt, dev, log):
    """The paper's ablations on the 12.6M-tet scene: every record layout under
    every curve order (time per pass, bytes per tet, the paper's Table 3, Table 4
    and Fig. 8 analogues), then primary walks from cameras at growing depth
    into the scene (visited tets per pixel and time, the Table 5 analogue).  The
    AO rays are built once, from the first configuration's primary hits."""
    import numpy as np
    import torch
    from synth import config_mesh, pinhole_rays, ao_rays, tri_geometry

    m = config_mesh("paper")
    o, d, _ = pinhole_rays((0.5, 0.5, 0.02), 1920, 1080, 60.0, tile=args.tile)
    po, pd = torch.from_numpy(o).to(dev), torch.from_numpy(d).to(dev)
    K = args.steps

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(K):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / K

    rows, ao_set = [], None
    for layout in ("tet20", "tet16", "tet32", "tet32n"):
        for sfc in ("hilbert", "hilbert_regions", "morton", "none"):
            t0 = time.time()
            mesh = tetrt.upload(m.points, m.tets, m.nbrs, m.cflag, layout=layout, sfc=sfc)
            up_s = time.time() - t0
            res = mesh.trace(po, pd, want_steps=True)
            if ao_set is None:
                tri = res["tri"].cpu().numpy()
                tp = res["t"].cpu().numpy()
                hit = tri >= 0
                hp = o[hit].astype(np.float64) + tp[hit, None].astype(np.float64) * d[hit].astype(np.float64)
                nrm, _ = tri_geometry(m.points, mesh.tri_vertices(tri[hit]))
                ao, ad, atm, parent = ao_rays(hp, nrm, d[hit], k=args.ao, seed=3, tmax=0.1)
                ao_set = [torch.from_numpy(x).to(dev) for x in (ao, ad, atm, tri[hit][parent].astype(np.int32))]
            A = ao_set
            out_p = tetrt.outputs(po.shape[0], dev)
            out_a = tetrt.outputs(A[0].shape[0], dev)
            ms_p = timed(lambda: mesh.trace_into(out_p, po, pd, block=args.block))
            ms_a = timed(lambda: mesh.trace_into(out_a, A[0], A[1], tmax=A[2], start_face=A[3], block=args.block))
            steps_p = float(res["steps"].double().mean().item())
            row = {"layout": layout, "sfc": sfc, "primary_ms": round(ms_p, 4), "ao_ms": round(ms_a, 4),
                   "mrays_s": round((po.shape[0] + A[0].shape[0]) / ((ms_p + ms_a) * 1e-3) / 1e6, 1),
                   "hot_bytes_per_tet": round(mesh.info["hot_bytes"] / m.n_tets, 2),
                   "all_bytes_per_tet": round((mesh.info["hot_bytes"] + mesh.info["cold_bytes"]) / m.n_tets, 2),
                   "primary_mean_steps": round(steps_p, 2), "upload_s": round(up_s, 2),
                   "regions": mesh.info["n_regions"]}
            log("ablate: %s" % json.dumps(row))
            rows.append(row)
            mesh.free()
    mesh = tetrt.upload(m.points, m.tets, m.nbrs, m.cflag, layout=args.layout, sfc=args.sfc)
    cams = []
    for z in (0.02, 0.1, 0.2, 0.3, 0.4):
        oc, dc, _ = pinhole_rays((0.5, 0.5, z), 1920, 1080, 60.0, tile=args.tile)
        oc, dc = torch.from_numpy(oc).to(dev), torch.from_numpy(dc).to(dev)
        res = mesh.trace(oc, dc, want_steps=True)
        out = tetrt.outputs(oc.shape[0], dev)
        ms = timed(lambda: mesh.trace_into(out, oc, dc, block=args.block))
        st = res["steps"].double()
        row = {"eye_z": z, "primary_ms": round(ms, 4), "mean_steps": round(float(st.mean().item()), 2),
               "hit_rate": round(float((res["tri"] >= 0).double().mean().item()), 4),
               "mrays_s": round(oc.shape[0] / (ms * 1e-3) / 1e6, 1)}
        log("ablate: %s" % json.dumps(row))
        cams.append(row)
    mesh.free()
    print(json.dumps({"metric": "ablations at 12.6M tets", "layouts_x_orders": rows, "camera_depth": cams,
                      "config": {"workload": "kuhn128-jitter0.1-20spheres, 1920x1080 + %d AO/hit" % args.ao,
                                 "steps": K, "block": args.block}}), flush=True)


def cpu_baseline(m, o, d, ao, ad, atm, sf, parent, hit, stride, threads, log):
    """The FP64 oracle on a strided sample of the same rays -- every ``stride``-th
    primary ray (started in the camera's tet, located once) and the AO rays
    generated from those rays' hits -- split into ``threads`` contiguous ranges
    traced concurrently (the oracle is reentrant and its C calls release the
    interpreter lock)."""
    import numpy as np
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    om = oracle.OracleMesh.from_kuhn(m)
    cam = om.locate(o[:1])
    sel = np.arange(0, o.shape[0], stride)
    hit_idx = np.nonzero(hit)[0]                     # primary index of each hit
    keep_hit = (hit_idx % stride) == 0
    sel_a = np.nonzero(keep_hit[parent])[0]
    po, pd = o[sel], d[sel]
    pst = np.full(sel.shape[0], cam[0], np.int32)
    A = (ao[sel_a], ad[sel_a], atm[sel_a], sf[sel_a])

    def pieces(n):
        b = np.linspace(0, n, threads + 1).astype(np.int64)
        return [(b[k], b[k + 1]) for k in range(threads) if b[k + 1] > b[k]]

    with ThreadPoolExecutor(threads) as ex:
        t0 = time.perf_counter()
        list(ex.map(lambda r: om.trace(po[r[0]:r[1]], pd[r[0]:r[1]], start_tet=pst[r[0]:r[1]]),
                    pieces(sel.shape[0])))
        t1 = time.perf_counter()
        list(ex.map(lambda r: om.trace(A[0][r[0]:r[1]], A[1][r[0]:r[1]], A[2][r[0]:r[1]],
                                       start_face=A[3][r[0]:r[1]]), pieces(sel_a.shape[0])))
        t2 = time.perf_counter()
    n = sel.shape[0] + sel_a.shape[0]
    log("oracle (%d threads): %d primary in %.1f s, %d AO in %.1f s" % (
        threads, sel.shape[0], t1 - t0, sel_a.shape[0], t2 - t1))
    # one thread on a smaller sample (every 64th of those primary rays and their AO rays)
    s1, s1a = slice(0, sel.shape[0], 64), np.nonzero(keep_hit[parent] & ((hit_idx[parent] % (64 * stride)) == 0))[0]
    t3 = time.perf_counter()
    om.trace(po[s1], pd[s1], start_tet=pst[s1])
    om.trace(ao[s1a], ad[s1a], atm[s1a], start_face=sf[s1a])
    t4 = time.perf_counter()
    n1 = po[s1].shape[0] + s1a.shape[0]
    return {"value": round(n / (t2 - t0) / 1e6, 4), "unit": "Mrays/s", "cores": threads, "kind": "oracle",
            "sample": "every %d-th primary ray (%d) + the AO rays of their hits (%d), %.1f s wall on %d "
                      "threads" % (stride, sel.shape[0], sel_a.shape[0], t2 - t0, threads),
            "single_thread_mrays_s": round(n1 / (t4 - t3) / 1e6, 4),
            "single_thread_sample": "%d primary + %d AO rays, %.1f s" % (po[s1].shape[0], s1a.shape[0], t4 - t3),
            "host_cpus": os.cpu_count(), "cpu": cpu_model()}


def cpu_model():
    """The host CPU's model name, as /proc/cpuinfo gives it."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


if __name__ == "__main__":
    main()
