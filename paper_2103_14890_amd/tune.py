"""Run the launch-shape autotuner on the batch workloads and store the choices.

    python -m paper_2103_14890_amd.tune [--out PATH] [--reps 5]

For each workload's plan (grid, kernel, precision, projection) the autotuner
of the library (qcoll_plan_autotune: tile family x cells per workgroup x grid
cap, timed with HIP events on the workload's own batch) picks a launch shape;
the shapes are written to a JSON cache keyed by the plan's shape, which
Plan.load_tuning() applies (by default from tuning_gfx950.json next to this
file). Needs a GPU.
"""

from __future__ import annotations

import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# (input batch, N, L, kernel, M, precisions, projection)
WORKLOADS = [
    ("hs2d_32", 32, 8.0, "hard_sphere", 8, ("fx16", "fp32"), True),
    ("hs2d_32", 32, 8.0, "hard_sphere", 8, ("fx16",), False),
    ("maxwell2d_32", 32, 8.0, "maxwell", 8, ("fx16", "fp32"), True),
    ("hs2d_64_noisy", 64, 10.0, "hard_sphere", 16, ("fx16", "fp32"), True),
    ("hs2d_64_noisy", 64, 10.0, "hard_sphere", 16, ("fx16",), False),
]


def main() -> int:
    import torch
    import workloads as wl
    from paper_2103_14890_amd import qcoll
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=qcoll.DEFAULT_TUNING)
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args()
    for name, N, L, kern, M, precs, conserve in WORKLOADS:
        f = torch.tensor(wl.config_inputs(name), dtype=torch.float32, device="cuda:0")
        for prec in precs:
            plan = qcoll.Plan(2, N, L, kern, M, precision=prec, conserve=conserve)
            best = plan.autotune(f, reps=args.reps, cache=args.out)
            print(f"{plan.key}: {best}", flush=True)
            plan.close()
        del f
    return 0


if __name__ == "__main__":
    sys.exit(main())
