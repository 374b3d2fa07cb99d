"""Write the oracle's full-size exact count of the 5-input 6x50 network (seed 0) as a fixture.

Workload: He-normal 5-50x6-5 ReLU network from seed 0, domain [0, 1]^5, unsafe iff
y0 - y1 > 0, maximum depth 40, leaf budget 2^20 (Alg. 1 with the level-boundary budget rule),
with the relaxation of Eq. 1 (one ratio, the default) or with one ratio per equation
(argument ``two``).
Calls only ``oracle/`` and the seeded input generator; nothing here comes from the HIP path.

Per level the fixture keeps the number of boxes, the class histogram, a SHA-256 digest of
the boxes' path ids and of their classes in canonical (path) order, and every box whose
decision margin is at most 1e-5 (depth, path, class, margin): a GPU count that differs from
the oracle anywhere can then be checked box by box against that list.

Usage: python tests/golden/make_acas_full.py [two]   (about 5 minutes on 8 cores)
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth                                    # noqa: E402
from oracle import count, slr                   # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
SMALL = 1e-5


def level_record(lev):
    order = np.argsort(lev["path"], kind="stable")
    path = lev["path"][order].astype("<u8")
    cls = lev["cls"][order].astype(np.int8)
    mg = slr.decision_margin(lev["g_lo"], lev["g_hi"])[order]
    small = np.nonzero(mg <= SMALL)[0]
    return dict(depth=int(lev["depth"]), n=int(path.size),
                n_unsafe=int(np.sum(cls == 1)), n_safe=int(np.sum(cls == 2)),
                n_undecided=int(np.sum(cls == 0)),
                path_sha256=hashlib.sha256(path.tobytes()).hexdigest(),
                cls_sha256=hashlib.sha256(cls.tobytes()).hexdigest(),
                small_margin=[[int(path[i]), int(cls[i]), float(mg[i])] for i in small])


def main(relax="one"):
    out_path = os.path.join(HERE, "acas0_d40_leaves2p20%s.json" % ("" if relax == "one" else "_two"))
    inst = synth.acas(0)
    t0 = time.time()
    r = count.count_exact(inst.net, inst.C, inst.dvec, inst.lo, inst.hi, 40, 1 << 20,
                          trace=True, chunk=16384, relax=relax)
    secs = time.time() - t0
    out = dict(
        workload="acas seed 0: 5-50x6-5 ReLU (He-normal), [0,1]^5, y0 - y1 > 0, D 40, 2^20 leaves"
                 + ("" if relax == "one" else ", two-ratio relaxation"),
        relax=relax,
        status=int(r["status"]), depth_reached=int(r["depth_reached"]),
        n_boxes_bounded=int(r["n_boxes_bounded"]), n_unsafe=int(r["n_unsafe"]),
        n_safe=int(r["n_safe"]), n_undecided=int(r["n_undecided"]),
        unsafe=r["unsafe"], safe=r["safe"], undecided=r["undecided"],
        unsafe_exact=str(r["unsafe_exact"]), safe_exact=str(r["safe_exact"]),
        undecided_exact=str(r["undecided_exact"]),
        hist_unsafe=[int(x) for x in r["hist_unsafe"]], hist_safe=[int(x) for x in r["hist_safe"]],
        hist_undecided=[int(x) for x in r["hist_undecided"]],
        small_margin_threshold=SMALL,
        levels=[level_record(lev) for lev in r["levels"]],
        oracle_seconds=round(secs, 1))
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {out_path}: {out['n_boxes_bounded']} boxes, depth {out['depth_reached']}, "
          f"{sum(len(l['small_margin']) for l in out['levels'])} small-margin boxes, {secs:.0f} s")


if __name__ == "__main__":
    main(*sys.argv[1:2])
