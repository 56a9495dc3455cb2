"""Python handle on the C oracle (``imin_oracle.c``).

TEST INFRASTRUCTURE ONLY: the oracle checks the GPU library and is loaded by
the tests, the smoke check and the CPU leg of the benchmark, never by the
library itself.  It is compiled with gcc into ``liboracle.so`` next to this
file; :func:`build` recompiles it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "imin_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

ALWAYS_LIVE = 0xFFFFFFFF
MODE_DOMINATOR = 0
MODE_DEFINITION = 1

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc -O2 (pthreads)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
                               "-pthread", "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        i32, i64, u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
        lib.oracle_philox4x32_10.argtypes = [P, P, P]
        lib.oracle_philox4x32_10.restype = None
        lib.oracle_thresholds.argtypes = [i64, P, P]
        lib.oracle_thresholds.restype = i64
        lib.oracle_coin.argtypes = [u64, u64, i64]
        lib.oracle_coin.restype = ctypes.c_uint32
        lib.oracle_eval.argtypes = [i32, i64, P, P, P, P, i32, P, u64, u64, u64, ctypes.c_int,
                                    ctypes.c_int, P, P, P, P]
        lib.oracle_eval.restype = ctypes.c_int
        lib.oracle_world.argtypes = [i32, i64, P, P, P, P, i32, P, u64, u64, ctypes.c_int, P, P]
        lib.oracle_world.restype = i32
        lib.oracle_solve.argtypes = [i32, i64, P, P, P, P, i32, i32, u64, u64, ctypes.c_int,
                                     ctypes.c_int, P, P, P, P]
        lib.oracle_solve.restype = ctypes.c_int
        lib.oracle_cp_world.argtypes = [i32, i64, P, P, P, P, i32, u64, u64, P, P, P, i64]
        lib.oracle_cp_world.restype = i32
        lib.oracle_max_coverage.argtypes = [i32, i64, P, P, P, P, i32, i32, u64, u64, ctypes.c_int,
                                            P, P, P, P, P]
        lib.oracle_max_coverage.restype = ctypes.c_int
        lib.oracle_coverage.argtypes = [i32, i64, P, P, P, P, i32, P, i32, u64, u64, ctypes.c_int, P]
        lib.oracle_coverage.restype = ctypes.c_int
        lib.oracle_reach_counts.argtypes = [i32, i64, P, P, P, P, i32, u64, u64, u64, ctypes.c_int, P]
        lib.oracle_reach_counts.restype = ctypes.c_int
        lib.oracle_world_sizes.argtypes = [i32, i64, P, P, P, P, i32, P, u64, u64, u64, ctypes.c_int, P]
        lib.oracle_world_sizes.restype = ctypes.c_int
        lib.oracle_cover_marginals.argtypes = [i32, i64, P, P, P, P, i32, P, i32, u64, u64, ctypes.c_int, P, P]
        lib.oracle_cover_marginals.restype = ctypes.c_int
        lib.oracle_lrr_pick.argtypes = [u64, u64, ctypes.c_uint32]
        lib.oracle_lrr_pick.restype = ctypes.c_uint32
        lib.oracle_lrr_set.argtypes = [i32, i64, P, P, P, P, i32, u64, u64, P, ctypes.c_uint32, P]
        lib.oracle_lrr_set.restype = i32
        lib.oracle_lrr_max_coverage.argtypes = [i32, i64, P, P, P, P, i32, P, ctypes.c_uint32, i32, u64, u64,
                                                ctypes.c_int, P, P, P, P, P]
        lib.oracle_lrr_max_coverage.restype = ctypes.c_int
        lib.oracle_lrr_coverage.argtypes = [i32, i64, P, P, P, P, i32, P, ctypes.c_uint32, P, i32, u64, u64,
                                            ctypes.c_int, P]
        lib.oracle_lrr_coverage.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def default_threads() -> int:
    return max(1, len(os.sched_getaffinity(0)))


def philox4x32_10(counter, key):
    """One Philox4x32-10 block: four uint32 words."""
    lib = _load()
    c = np.asarray(counter, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    lib.oracle_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def coin(seed: int, w: int, e: int) -> int:
    return int(_load().oracle_coin(seed, w, e))


def thresholds(p) -> np.ndarray:
    """uint32 coin thresholds; raises ValueError on p outside [0, 1] or NaN."""
    lib = _load()
    p = np.ascontiguousarray(p, dtype=np.float32)
    thr = np.zeros(p.shape[0], dtype=np.uint32)
    bad = lib.oracle_thresholds(p.shape[0], _ptr(p), _ptr(thr))
    if bad >= 0:
        raise ValueError(f"edge {bad}: probability {p[bad]!r} is not in [0, 1]")
    return thr


class Query:
    """A graph plus seed set, with thresholds computed once."""

    def __init__(self, g, seeds):
        self.n = int(g.n)
        self.m = int(g.m)
        self.row_ptr = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
        self.col = np.ascontiguousarray(g.col, dtype=np.int32)
        self.thr = thresholds(g.p)
        self.seeds = np.ascontiguousarray(seeds, dtype=np.int32)

    def _blocked(self, blocked):
        if blocked is None:
            return None
        b = np.zeros(self.n, dtype=np.uint8)
        b[np.asarray(list(blocked), dtype=np.int64)] = 1
        return b

    def eval(self, rng_seed: int, w0: int, nw: int, blocked=(), mode: int = MODE_DOMINATOR,
             threads: int | None = None, per_world: bool = False):
        """gain int64[n] and total over worlds [w0, w0+nw) under ``blocked``."""
        lib = _load()
        blk = self._blocked(blocked)
        gain = np.zeros(self.n, dtype=np.int64)
        total = np.zeros(1, dtype=np.int64)
        rsize = np.zeros(nw, dtype=np.int32) if per_world else None
        rsum = np.zeros(nw, dtype=np.int64) if per_world else None
        st = lib.oracle_eval(self.n, self.m, _ptr(self.row_ptr), _ptr(self.col), _ptr(self.thr),
                             _ptr(self.seeds), len(self.seeds), _ptr(blk), rng_seed, w0, nw, mode,
                             threads or default_threads(), _ptr(gain), _ptr(total), _ptr(rsize),
                             _ptr(rsum))
        if st != 0:
            raise ValueError("oracle_eval rejected the query")
        if per_world:
            return gain, int(total[0]), rsize, rsum
        return gain, int(total[0])

    def world(self, rng_seed: int, w: int, blocked=(), mode: int = MODE_DOMINATOR):
        """(c int32[n], reached list in BFS order) for one world."""
        lib = _load()
        blk = self._blocked(blocked)
        c = np.zeros(self.n, dtype=np.int32)
        reached = np.zeros(self.n, dtype=np.int32)
        R = lib.oracle_world(self.n, self.m, _ptr(self.row_ptr), _ptr(self.col), _ptr(self.thr),
                             _ptr(self.seeds), len(self.seeds), _ptr(blk), rng_seed, w, mode,
                             _ptr(c), _ptr(reached))
        if R < 0:
            raise ValueError("oracle_world rejected the query")
        return c, reached[:R].copy()

    def solve(self, k: int, theta: int, rng_seed: int, mode: int = MODE_DOMINATOR,
              threads: int | None = None):
        """Greedy selection; returns dict(blockers, gains, spread_totals, n_selected)."""
        lib = _load()
        blockers = np.zeros(max(k, 1), dtype=np.int32)
        gains = np.zeros(max(k, 1), dtype=np.int64)
        totals = np.zeros(k + 1, dtype=np.int64)
        nsel = np.zeros(1, dtype=np.int32)
        st = lib.oracle_solve(self.n, self.m, _ptr(self.row_ptr), _ptr(self.col), _ptr(self.thr),
                              _ptr(self.seeds), len(self.seeds), k, theta, rng_seed, mode,
                              threads or default_threads(), _ptr(blockers), _ptr(gains),
                              _ptr(totals), _ptr(nsel))
        if st != 0:
            raise ValueError("oracle_solve rejected the query")
        r = int(nsel[0])
        return dict(blockers=blockers[:r].copy(), gains=gains[:r].copy(),
                    spread_totals=totals[:r + 1].copy(), n_selected=r)

    # ---------------------------------------------------------- coverage
    def cp_world(self, rng_seed: int, w: int):
        """The CP sequence of world w (Definition 4.1, Algorithm 2): a list of
        (node, CP set) in depth-first preorder from the virtual source."""
        lib = _load()
        node = np.zeros(self.n, dtype=np.int32)
        off = np.zeros(self.n + 1, dtype=np.int64)
        cap = 1 << 16
        while True:
            cp = np.zeros(cap, dtype=np.int32)
            ne = lib.oracle_cp_world(self.n, self.m, _ptr(self.row_ptr), _ptr(self.col), _ptr(self.thr),
                                     _ptr(self.seeds), len(self.seeds), rng_seed, w, _ptr(node), _ptr(off),
                                     _ptr(cp), cap)
            if ne == -2:
                cap *= 4
                continue
            if ne < 0:
                raise ValueError("oracle_cp_world rejected the query")
            return [(int(node[i]), [int(x) for x in cp[off[i]:off[i + 1]]]) for i in range(ne)]

    def max_coverage(self, k: int, theta: int, rng_seed: int, threads: int | None = None):
        """Max-Coverage over the CP sequences of worlds [0, theta): dict(blockers,
        gains, cov, cov_upper, n_selected); cov and cov_upper have n_selected+1
        entries (every prefix B_0 .. B_{n_selected})."""
        lib = _load()
        blockers = np.zeros(max(k, 1), dtype=np.int32)
        gains = np.zeros(max(k, 1), dtype=np.int64)
        cov = np.zeros(k + 1, dtype=np.int64)
        cu = np.zeros(k + 1, dtype=np.int64)
        nsel = np.zeros(1, dtype=np.int32)
        st = lib.oracle_max_coverage(self.n, self.m, _ptr(self.row_ptr), _ptr(self.col), _ptr(self.thr),
                                     _ptr(self.seeds), len(self.seeds), k, theta, rng_seed,
                                     threads or default_threads(), _ptr(blockers), _ptr(gains), _ptr(cov),
                                     _ptr(cu), _ptr(nsel))
        if st != 0:
            raise ValueError("oracle_max_coverage rejected the query")
        r = int(nsel[0])
        return dict(blockers=blockers[:r].copy(), gains=gains[:r].copy(), cov=cov[:r + 1].copy(),
                    cov_upper=cu[:r + 1].copy(), n_selected=r)

    def coverage(self, blockers, theta: int, rng_seed: int, threads: int | None = None) -> int:
        """Cov(B) over the CP sequences of worlds [0, theta) (Section 4.1)."""
        lib = _load()
        b = np.ascontiguousarray(blockers, dtype=np.int32)
        out = np.zeros(1, dtype=np.int64)
        st = lib.oracle_coverage(self.n, self.m, _ptr(self.row_ptr), _ptr(self.col), _ptr(self.thr),
                                 _ptr(self.seeds), len(self.seeds), _ptr(b), len(b), theta, rng_seed,
                                 threads or default_threads(), _ptr(out))
        if st != 0:
            raise ValueError("oracle_coverage rejected the query")
        return int(out[0])

    def reach_counts(self, rng_seed: int, w0: int, nw: int, threads: int | None = None) -> np.ndarray:
        """int64[n]: in how many worlds of [w0, w0+nw) each node is reached."""
        lib = _load()
        out = np.zeros(self.n, dtype=np.int64)
        st = lib.oracle_reach_counts(self.n, self.m, _ptr(self.row_ptr), _ptr(self.col), _ptr(self.thr),
                                     _ptr(self.seeds), len(self.seeds), rng_seed, w0, nw,
                                     threads or default_threads(), _ptr(out))
        if st != 0:
            raise ValueError("oracle_reach_counts rejected the query")
        return out

    def world_sizes(self, rng_seed: int, w0: int, nw: int, threads: int | None = None,
                    blocked=()) -> np.ndarray:
        """int32[nw]: |R_w(B)| of worlds [w0, w0+nw) with the blockers B."""
        lib = _load()
        blk = self._blocked(blocked) if len(blocked) else None
        out = np.zeros(nw, dtype=np.int32)
        st = lib.oracle_world_sizes(self.n, self.m, _ptr(self.row_ptr), _ptr(self.col), _ptr(self.thr),
                                    _ptr(self.seeds), len(self.seeds), _ptr(blk), rng_seed, w0, nw,
                                    threads or default_threads(), _ptr(out))
        if st != 0:
            raise ValueError("oracle_world_sizes rejected the query")
        return out

    def cover_marginals(self, blockers, theta: int, rng_seed: int, threads: int | None = None):
        """(marg int64[n], Cov(B)): the marginal coverage of every node given B
        (0 on B and the seeds) over the CP sequences of worlds [0, theta)."""
        lib = _load()
        b = np.ascontiguousarray(blockers, dtype=np.int32)
        marg = np.zeros(self.n, dtype=np.int64)
        cov = np.zeros(1, dtype=np.int64)
        st = lib.oracle_cover_marginals(self.n, self.m, _ptr(self.row_ptr), _ptr(self.col), _ptr(self.thr),
                                        _ptr(self.seeds), len(self.seeds), _ptr(b), len(b), theta, rng_seed,
                                        threads or default_threads(), _ptr(marg), _ptr(cov))
        if st != 0:
            raise ValueError("oracle_cover_marginals rejected the query")
        return marg, int(cov[0])

    # ----------------------------------------------------- global sampling
    def lrr_set(self, key: int, i: int, vprime) -> list:
        """The LRR set of sample i (Algorithm 3): sorted members, [] when empty."""
        lib = _load()
        vp = np.ascontiguousarray(vprime, dtype=np.int32)
        out = np.zeros(self.n, dtype=np.int32)
        r = lib.oracle_lrr_set(self.n, self.m, _ptr(self.row_ptr), _ptr(self.col), _ptr(self.thr),
                               _ptr(self.seeds), len(self.seeds), key, i, _ptr(vp), len(vp), _ptr(out))
        if r < 0:
            raise ValueError("oracle_lrr_set rejected the query")
        return sorted(int(x) for x in out[:r])

    def lrr_max_coverage(self, vprime, k: int, theta: int, key: int, threads: int | None = None):
        """Max-Coverage over the LRR sets of samples [0, theta); as max_coverage."""
        lib = _load()
        vp = np.ascontiguousarray(vprime, dtype=np.int32)
        blockers = np.zeros(max(k, 1), dtype=np.int32)
        gains = np.zeros(max(k, 1), dtype=np.int64)
        cov = np.zeros(k + 1, dtype=np.int64)
        cu = np.zeros(k + 1, dtype=np.int64)
        nsel = np.zeros(1, dtype=np.int32)
        st = lib.oracle_lrr_max_coverage(self.n, self.m, _ptr(self.row_ptr), _ptr(self.col), _ptr(self.thr),
                                         _ptr(self.seeds), len(self.seeds), _ptr(vp), len(vp), k, theta, key,
                                         threads or default_threads(), _ptr(blockers), _ptr(gains), _ptr(cov),
                                         _ptr(cu), _ptr(nsel))
        if st != 0:
            raise ValueError("oracle_lrr_max_coverage rejected the query")
        r = int(nsel[0])
        return dict(blockers=blockers[:r].copy(), gains=gains[:r].copy(), cov=cov[:r + 1].copy(),
                    cov_upper=cu[:r + 1].copy(), n_selected=r)

    def lrr_coverage(self, vprime, blockers, theta: int, key: int, threads: int | None = None) -> int:
        """Cov(B) over the LRR sets of samples [0, theta)."""
        lib = _load()
        vp = np.ascontiguousarray(vprime, dtype=np.int32)
        b = np.ascontiguousarray(blockers, dtype=np.int32)
        out = np.zeros(1, dtype=np.int64)
        st = lib.oracle_lrr_coverage(self.n, self.m, _ptr(self.row_ptr), _ptr(self.col), _ptr(self.thr),
                                     _ptr(self.seeds), len(self.seeds), _ptr(vp), len(vp), _ptr(b), len(b),
                                     theta, key, threads or default_threads(), _ptr(out))
        if st != 0:
            raise ValueError("oracle_lrr_coverage rejected the query")
        return int(out[0])


def lrr_pick(key: int, i: int, nvp: int) -> int:
    """Index into V'_s of sample i's target (Algorithm 3)."""
    return int(_load().oracle_lrr_pick(key, i, nvp))
