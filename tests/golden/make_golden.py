"""Write tests/golden/cube_lattice_10_substeps.json: summary values of the
FP64 oracle on the plain cube-lattice scene (4,096 particles, 32^3 grid,
fixed corotated E = 1e5, nu = 0.3, dt = 1e-4) after 10 substeps.

Calls only the oracle (and the seeded input generator).  Re-run only when
the oracle's arithmetic changes for a reason named in the commit message.
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import mpm_oracle as O  # noqa: E402
from paper_2602_01723_amd import scenes  # noqa: E402

STEPS = 10
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cube_lattice_10_substeps.json")


def summary():
    sc = scenes.make_scene("cube_lattice")
    p = O.Params.from_scene(sc)
    x, v, C, F = O.step_n(O.state_from_scene(sc), p, STEPS)
    m = p.mass
    eye = __import__("torch").eye(3, dtype=F.dtype)
    return {
        "scene": "cube_lattice (seed 0, 4096 particles, 32^3, dt 1e-4)",
        "substeps": STEPS,
        "total_mass": float(m.sum()),
        "centre_of_mass": [float(c) for c in (m[:, None] * x).sum(0) / m.sum()],
        "momentum": [float(c) for c in (m[:, None] * v).sum(0)],
        "mean_abs_F_minus_I": float((F - eye).abs().mean()),
        "max_abs_C": float(C.abs().max()),
        "x_first_particles": [[float(a) for a in row] for row in x[:4]],
    }


if __name__ == "__main__":
    with open(OUT, "w") as fh:
        json.dump(summary(), fh, indent=1)
    print("wrote", OUT)
