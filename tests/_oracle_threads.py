"""The oracle over contiguous ray ranges in threads, for tests at large sizes
(its C calls release the interpreter lock; the results are those of one call)."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np


def oracle_trace(om, o, d, tmax=None, start_face=None, start_tet=None, threads=16):
    n = o.shape[0]
    cuts = np.linspace(0, n, threads + 1).astype(int)
    parts = [(a, b) for a, b in zip(cuts[:-1], cuts[1:]) if b > a]
    if not parts:
        return om.trace(o, d, tmax, start_face=start_face, start_tet=start_tet)

    def cut(x, a, b):
        return None if x is None else x[a:b]

    def run(ab):
        a, b = ab
        return om.trace(o[a:b], d[a:b], cut(tmax, a, b), start_face=cut(start_face, a, b),
                        start_tet=cut(start_tet, a, b))

    with ThreadPoolExecutor(len(parts)) as ex:
        res = list(ex.map(run, parts))
    return {k: np.concatenate([r[k] for r in res]) for k in res[0]}
