"""Compute and cache the host eigenvalues the benchmark configurations draw
their shifts from (LAPACK via scipy; minutes for the n=8000 case).

Usage: python -m workloads.make_cache [c2] [c3] [c4] [c5]
"""
import sys
import time

from workloads import generators as g


def main(argv):
    which = argv or ["c2", "c3", "c4", "c5"]
    for w in which:
        t = time.time()
        if w == "c2":
            g.config_c2()
        elif w == "c3":
            g.config_c3(grade=False)
        elif w == "c4":
            g.config_c4()
        elif w == "c5":
            g.config_c5_pool()
        print(f"{w}: {time.time() - t:.1f} s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
