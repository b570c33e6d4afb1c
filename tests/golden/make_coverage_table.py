"""Writes coverage_e01.txt: reference counts and coverage statistics of the
reference schedules (section Experiments, Shift Schedule Analysis: the
coverage map C(x), its mean, standard deviation and coefficient of
variation) on the workload shapes, computed by the oracle alone.

Usage: python tests/golden/make_coverage_table.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402

# (name, shape, patch, step): the workloads' shapes, plus the 2-D image
# shapes of the schedule analysis' test images (shapes only)
SHAPES = [
    ("image-128", (128, 128), (8, 8), (3, 3)),
    ("image-256", (256, 256), (8, 8), (3, 3)),
    ("image-512", (512, 512), (8, 8), (3, 3)),
    ("image-481x321", (481, 321), (8, 8), (3, 3)),
    ("image-768x512", (768, 512), (8, 8), (3, 3)),
    ("microscopy-1024", (1024, 1024), (8, 8), (3, 3)),
    ("phantom-256x256x128", (256, 256, 128), (4, 4, 4), (3, 3, 3)),
    ("ecg-65536", (65536,), (32,), (4,)),
]
# (schedule, shift density rho_s, schedule density K_s)
SCHEDULES = [("off", 0.0, 1)] + [(s, r, k) for s in ("generated", "balanced")
                                 for r, k in ((1.0, 1), (1.0, 2), (2.0, 1), (2.0, 2), (4.0, 2))] \
    + [("sparse", 2.0, 2)]


def rows():
    for name, shape, patch, step in SHAPES:
        for sched, rho, ks in SCHEDULES:
            st = O.Stage(shape=shape, patch=patch, step=step, search=(1,) * len(shape),
                         schedule=sched, shift_density=rho, passes=ks)
            n = len(O.schedule(st))
            _, mean, sd, cv = O.coverage(st)
            yield name, sched, rho, ks, n, mean, sd, cv


def main():
    out = os.path.join(HERE, "coverage_e01.txt")
    with open(out, "w") as f:
        f.write("# Reference counts and coverage statistics of the reference schedules\n"
                "# (section Experiments, Shift Schedule Analysis), written by\n"
                "# make_coverage_table.py from the oracle alone.\n"
                "# name schedule rho_s K_s n_refs mean_C std_C cv_C\n")
        for name, sched, rho, ks, n, mean, sd, cv in rows():
            f.write(f"{name} {sched} {rho:g} {ks} {n} {mean:.17g} {sd:.17g} {cv:.17g}\n")
    print("wrote", out)


if __name__ == "__main__":
    main()
