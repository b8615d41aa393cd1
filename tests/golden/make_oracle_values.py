"""Write oracle_converged.json: converged costs E* of the parity scenes.

Calls only the oracle (FP64 LM with exact Schur solves) on the seeded
scenes; the GPU tests compare their converged cost with these values.
Run from the repository root:
    python tests/golden/make_oracle_values.py [scene names]
With names, only those entries are recomputed (the 200-camera scene takes
about 40 s per LM iteration on 8 cores); without, every scene.
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from scenegen import make_scene, small_config, manhattan_config  # noqa: E402
from oracle import lm  # noqa: E402

SCENES = {
    "tiny_holistic": lambda: make_scene(small_config(n_cams=9, n_points=70, n_lines=20), seed=101),
    "points_10cam": lambda: make_scene(1),
    "holistic_30cam": lambda: make_scene(2),
    "holistic_200cam": lambda: make_scene(3),
    "manhattan_relations": lambda: make_scene(manhattan_config(), seed=12),
}

if __name__ == "__main__":
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_converged.json")
    names = sys.argv[1:] or list(SCENES)
    out = json.load(open(path)) if os.path.exists(path) else {}
    for name in names:
        t = time.time()
        prob = lm.Problem(SCENES[name]())
        res = lm.lm_solve(prob, func_tol=1e-12, max_iters=200, verbose=name == "holistic_200cam")
        out[name] = dict(E=res["E"], Epix=res["Epix"], iters=res["iters"], accepted=res["accepted"],
                         reason=res["reason"], seconds=round(time.time() - t, 1))
        print(name, out[name], flush=True)
        with open(path, "w") as f:
            json.dump(out, f, indent=1)
