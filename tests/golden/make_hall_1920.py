"""Writes ``hall_1920_seed0.npz`` beside this script: the FP64 oracle's
densification of the 1920x960 hall keyframe (scene seed 0, PatchMatch seed 0)
with the workload's configured parameters -- 4 neighbours, 11x11 patch
sampled every 2nd pixel (36 samples), 8 red-black iterations with 6
refinement trials, 0.3-30 m -- before and after the geometric-consistency
step (Sec. III, densification thread) against the four neighbours' rendered
range maps (1 px, 1%, at least 2 agreeing maps).

It calls only ``oracle`` and ``synth``; nothing here comes from the HIP path.
On 8 host cores it takes about ten minutes.

Stored (all (H, W) unless noted):

* ``depth_code`` uint16: 0 where the oracle's PatchMatch result is invalid,
  else 1 + round((ln d - ln d_min) / (ln d_max - ln d_min) * 65534), i.e.
  the range on a log scale with a relative step of 7.0e-5 (decoding error
  <= 3.6e-5 relative, 1/140 of the 0.5% parity bar);
* ``cost_code`` uint16: round(cost / 2 * 65535) (step 3.1e-5, 1/6 of the
  2e-4 quality bar), cost 2 = invalid;
* ``keep_bits`` uint8: ``numpy.packbits`` of the pixels the consistency
  step keeps (row-major, H*W bits);
* ``meta`` (JSON string): sizes, seeds, parameters, range-code limits,
  SHA-256 of the oracle's and the renderer's C sources, wall time, threads.

Run from the repository root: ``python tests/golden/make_hall_1920.py``.
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(HERE, "hall_1920_seed0.npz")
CODE_MAX = 65534


def source_hash() -> str:
    h = hashlib.sha256()
    for p in (os.path.join(ROOT, "oracle", "pmsref.c"), os.path.join(ROOT, "oracle", "pmsref.h"),
              os.path.join(ROOT, "synth", "render.c")):
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def encode_depth(d, dmin, dmax):
    code = np.zeros(d.shape, dtype=np.uint16)
    v = d > 0
    s = (np.log(d[v]) - np.log(dmin)) / (np.log(dmax) - np.log(dmin))
    code[v] = 1 + np.rint(np.clip(s, 0.0, 1.0) * CODE_MAX).astype(np.uint16)
    return code


def encode_cost(c):
    return np.rint(np.clip(c, 0.0, 2.0) / 2.0 * 65535).astype(np.uint16)


def main() -> None:
    w = synth.workload("hall_1920", seed=0)
    p = dict(w.params)
    imgs = [np.asarray(a, dtype=np.float64) for a in w.images_f32()]
    ref, nbrs = imgs[w.ref], [imgs[i] for i in w.nbrs]
    rp, nps = w.poses[w.ref], [w.poses[i] for i in w.nbrs]
    maps = [w.gt_depth[i].astype(np.float64) for i in w.maps]
    mposes = [w.poses[i] for i in w.maps]
    threads = os.cpu_count() or 1
    print(f"oracle densify hall_1920 {w.W}x{w.H}, {len(nbrs)} views, "
          f"{p['iterations']} iterations on {threads} threads", flush=True)
    t0 = time.time()
    d, n, c = oracle.densify(ref, nbrs, rp, nps, p, n_threads=threads)
    t1 = time.time()
    print(f"patchmatch {t1 - t0:.0f} s", flush=True)
    dk, _, _ = oracle.consistency(d, n, c, rp, maps, mposes, p, n_threads=threads)
    keep = dk > 0
    print(f"valid {(d > 0).mean():.4f}, kept {keep.mean():.4f}", flush=True)
    meta = dict(workload="hall_1920", scene_seed=0, W=w.W, H=w.H, ref=w.ref, nbrs=w.nbrs,
                maps=w.maps, params={k: v for k, v in p.items()},
                depth_code=dict(d_min=p["depth_min"], d_max=p["depth_max"], code_max=CODE_MAX),
                sources_sha256=source_hash(), patchmatch_wall_s=round(t1 - t0, 1),
                threads=threads)
    np.savez_compressed(OUT, depth_code=encode_depth(d, p["depth_min"], p["depth_max"]),
                        cost_code=encode_cost(c), keep_bits=np.packbits(keep.reshape(-1)),
                        meta=np.array(json.dumps(meta)))
    print(f"wrote {OUT} ({os.path.getsize(OUT) / 2**20:.2f} MiB)", flush=True)


if __name__ == "__main__":
    main()
