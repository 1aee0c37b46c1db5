#!/usr/bin/env python3
"""Closest-hit throughput on the 12.6M-tet scene (one MI355X).

Workload: the unit cube as a 128^3 Kuhn grid (12,582,912 tets, 2,146,689
points, interior vertices jittered by +-0.1 cell), constrained faces on the
boundary of a union of 20 seeded spheres; 1920x1080 primary rays from a camera
at (0.5, 0.5, 0.02) looking +z with a 60 degree horizontal field of view
(emitted in 8x8 pixel tiles), then 8 cosine-weighted ambient-occlusion rays
(tmax 0.1) from every primary hit.  The AO ray set is built once, before
timing, from the library's own primary hits.

One step = trace_closest on all primary rays (each locates its origin on the
device) + trace_closest on all AO rays (each starts from its hit face).  Inputs
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
    ap.add_argument("--workload", default="paper", choices=["paper", "tiny"])
    ap.add_argument("--tile", type=int, default=8, help="pixel tile edge for ray order (1 = row-major)")
    ap.add_argument("--sfc", default="hilbert", choices=["hilbert", "morton", "none"])
    ap.add_argument("--layout", default="tet16", choices=["tet20", "tet16", "tet32n"])
    ap.add_argument("--block", type=int, default=256)
    ap.add_argument("--kernel", type=int, default=0, help="0 auto, 1 one lane per ray, 2 persistent")
    ap.add_argument("--refill", type=int, default=0, help="persistent refill threshold (0 = default)")
    ap.add_argument("--ao", type=int, default=8, help="AO rays per primary hit")
    ap.add_argument("--sort", type=int, default=0, help="ray binning: 0 auto, 1 off, 2 on")
    ap.add_argument("--sort-chunk", type=int, default=0, help="log2 rays per binning chunk (0 = default)")
    ap.add_argument("--sort-dirq", type=int, default=0, help="direction bins per axis (0 = default)")
    ap.add_argument("--sort-cells", type=int, default=0, help="log2 origin cells per axis (0 = default)")
    ap.add_argument("--eye", default="", help="camera position x,y,z (default: the workload's)")
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--cpu-stride", type=int, default=4,
                    help="oracle sample: every n-th primary ray and the AO rays of its hits")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run a device copy of this size (counter calibration runs)")
    return ap.parse_args()


def workload(name):
    from synth import config_mesh
    if name == "paper":
        return config_mesh("paper"), (0.5, 0.5, 0.02), 1920, 1080
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

    # set-up pass (untimed): primary hits -> AO rays, step counts for the byte model
    res = mesh.trace(po, pd, want_steps=True)
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

    kw = dict(block=args.block, kernel=args.kernel, refill=args.refill, sort=args.sort,
              sort_chunk_log2=args.sort_chunk, sort_dirq=args.sort_dirq,
              sort_cells_log2=args.sort_cells)

    def step():
        mesh.trace_into(out_p, po, pd, **kw)
        mesh.trace_into(out_a, ao_t, ad_t, tmax=atm_t, start_face=sf_t, **kw)

    for _ in range(args.warmup):
        step()
    if args.copy_probe_mib > 0:
        nbytes = args.copy_probe_mib << 20
        src = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy probe: %d bytes read, %d bytes written" % (nbytes, nbytes))
        del src, dst
    torch.cuda.synchronize()

    K = args.steps
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(K)]
    t_wall = time.perf_counter()
    for k in range(K):
        ev[k][0].record()
        mesh.trace_into(out_p, po, pd, **kw)
        ev[k][1].record()
        mesh.trace_into(out_a, ao_t, ad_t, tmax=atm_t, start_face=sf_t, **kw)
        ev[k][2].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    ms_p = np.array([ev[k][0].elapsed_time(ev[k][1]) for k in range(K)])
    ms_a = np.array([ev[k][1].elapsed_time(ev[k][2]) for k in range(K)])
    ms_step = float(ev[0][0].elapsed_time(ev[K - 1][2]) / K)
    rays = n_p + n_a
    value = rays / (ms_step * 1e-3) / 1e6

    # algorithmic bytes per launch: per-ray I/O plus 20 B per walk step
    bytes_p = int(steps_p.sum()) * STEP_BYTES + n_p * RAY_IO_BYTES
    bytes_a = int(steps_a.sum()) * STEP_BYTES + n_a * (RAY_IO_BYTES + 2 * OPT_INPUT_BYTES)
    kern = {"primary": (ms_p.mean(), bytes_p, n_p), "ao": (ms_a.mean(), bytes_a, n_a)}
    dom = max(kern, key=lambda k: kern[k][0])
    dom_ms, dom_bytes, dom_rays = kern[dom]
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9

    line = {
        "metric": "closest-hit Mrays/s at 12.6M tets",
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
            "workload": ("kuhn128-jitter0.1-20spheres, 1920x1080 primary + %d AO/hit (tmax 0.1)" % args.ao
                         if args.workload == "paper" else "kuhn16-sphere, 64x64 primary + %d AO/hit" % args.ao),
            "tets": m.n_tets, "points": m.n_points, "triangles": info["n_tris"],
            "primary_rays": n_p, "ao_rays": n_a, "ray_order": "8x8 tiles" if args.tile == 8 else
            ("row-major" if args.tile <= 1 else "%dx%d tiles" % (args.tile, args.tile)),
            "layout": args.layout, "sfc": args.sfc, "block": args.block,
            "kernel": {0: "auto", 1: "one lane per ray", 2: "persistent lanes"}[args.kernel],
            "ray_binning": {0: "auto", 1: "off", 2: "on"}[args.sort], "eye": list(eye),
        },
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": "k_trace (%s rays)" % dom, "kernel_ms": round(float(dom_ms), 4),
            "algorithmic_bytes": dom_bytes,
        },
        "detail": {
            "primary_ms": round(float(ms_p.mean()), 4), "ao_ms": round(float(ms_a.mean()), 4),
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
        line["cpu_baseline"] = cpu_baseline(m, o, d, ao, ad, atm, sf, parent, hit, args.cpu_stride, log)
    mesh.free()
    print(json.dumps(line), flush=True)


def cpu_baseline(m, o, d, ao, ad, atm, sf, parent, hit, stride, log):
    """The FP64 oracle, single-threaded, on a strided sample of the same rays:
    every ``stride``-th primary ray (started in the camera's tet, located once)
    and the AO rays generated from those rays' hits."""
    import numpy as np
    import oracle
    om = oracle.OracleMesh.from_kuhn(m)
    cam = om.locate(o[:1])
    sel = np.arange(0, o.shape[0], stride)
    hit_idx = np.nonzero(hit)[0]                     # primary index of each hit
    keep_hit = (hit_idx % stride) == 0
    sel_a = np.nonzero(keep_hit[parent])[0]
    t0 = time.perf_counter()
    om.trace(o[sel], d[sel], start_tet=np.full(sel.shape[0], cam[0], np.int32))
    t1 = time.perf_counter()
    om.trace(ao[sel_a], ad[sel_a], atm[sel_a], start_face=sf[sel_a])
    t2 = time.perf_counter()
    n = sel.shape[0] + sel_a.shape[0]
    log("oracle: %d primary in %.1f s, %d AO in %.1f s" % (sel.shape[0], t1 - t0, sel_a.shape[0], t2 - t1))
    return {"value": round(n / (t2 - t0) / 1e6, 4), "unit": "Mrays/s", "cores": 1, "kind": "oracle",
            "sample": "every %d-th primary ray (%d) + the AO rays of their hits (%d), %.1f s" % (
                stride, sel.shape[0], sel_a.shape[0], t2 - t0)}


if __name__ == "__main__":
    main()
