"""The oracle render over many rays in a pool of worker processes (TEST INFRASTRUCTURE).

``oracle_render`` is plain and single-threaded in its placement; a full
1920x1080 frame is ~2 M rays, so the parity tests and the CPU baseline split
the rays into chunks and render them in spawned worker processes.  The
scene, the rays and any per-ray arrays to compare against are shared
through memory-mapped files (a temporary directory, /dev/shm when present),
so the workers start clean (no copy of the parent's state, no device
context) and nothing large is pickled.  The arithmetic is exactly
``oracle_render``'s; only the work is split.
"""
from __future__ import annotations

import multiprocessing as mp
import os
import shutil
import tempfile
import time
from typing import Callable, Dict, Optional

import numpy as np

_W: dict = {}


def _share(arr: np.ndarray, path: str) -> dict:
    a = np.ascontiguousarray(arr)
    mm = np.lib.format.open_memmap(path, mode="w+", dtype=a.dtype, shape=a.shape)
    mm[...] = a
    mm.flush()
    del mm
    return {"path": path}


def _load(spec: dict):
    return np.load(spec["path"], mmap_mode="r")


def _init(spec: dict) -> None:
    import torch

    torch.set_num_threads(1)
    _W["scene"] = {k: (_load(v) if isinstance(v, dict) else v) for k, v in spec["scene"].items()}
    _W["o"] = _load(spec["o"])
    _W["d"] = _load(spec["d"])
    _W["cmp"] = {k: _load(v) for k, v in spec["cmp"].items()}
    _W["prm"] = spec["prm"]


def _work(rng):
    from .render import oracle_render

    a, b = rng
    keep_k = "k_list" in _W["cmp"]
    res = oracle_render(_W["scene"], np.asarray(_W["o"][a:b]), np.asarray(_W["d"][a:b]), _W["prm"], keep_k=keep_k)
    out = {k: res[k] for k in ("C", "T", "F", "n_placed", "n_eval")}
    if keep_k:
        got = np.asarray(_W["cmp"]["k_list"][a:b])
        bad = np.nonzero(np.any(got != res["k_list"], axis=1))[0]
        out["k_mismatch_rays"] = (bad + a).astype(np.int64)
    return a, b, out


def render_parallel(scene: Dict[str, np.ndarray], o: np.ndarray, d: np.ndarray, prm, workers: Optional[int] = None,
                    chunk: int = 8192, k_list: Optional[np.ndarray] = None,
                    log: Optional[Callable[[str], None]] = None) -> dict:
    """oracle_render of rays (o, d) split into chunks over `workers`
    processes (default: the CPUs this process may run on, at most 16).

    Returns float64 C [n, 3], T [n], F [n, 7], int32 n_placed, n_eval [n],
    'workers' and 'seconds'; with k_list (the [n, n_max] lattice indices to
    check, -1 padded) also 'k_mismatch_rays', the rays whose k-list differs
    from the oracle's."""
    n = o.shape[0]
    if workers is None:
        workers = min(16, len(os.sched_getaffinity(0)))
    base = "/dev/shm" if os.path.isdir("/dev/shm") else None
    tmp = tempfile.mkdtemp(prefix="oracle_pool_", dir=base)
    try:
        spec = {"scene": {}, "cmp": {}, "prm": prm}
        for k, v in scene.items():
            spec["scene"][k] = _share(v, os.path.join(tmp, f"scene_{k}.npy")) if isinstance(v, np.ndarray) \
                and v.size > 64 else v
        spec["o"] = _share(np.asarray(o, np.float32), os.path.join(tmp, "o.npy"))
        spec["d"] = _share(np.asarray(d, np.float32), os.path.join(tmp, "d.npy"))
        if k_list is not None:
            spec["cmp"]["k_list"] = _share(np.asarray(k_list, np.int32), os.path.join(tmp, "k_list.npy"))
        out = {"C": np.zeros((n, 3)), "T": np.zeros(n), "F": np.zeros((n, 7)),
               "n_placed": np.zeros(n, np.int32), "n_eval": np.zeros(n, np.int32)}
        bad = []
        t0 = time.time()
        ranges = [(a, min(n, a + chunk)) for a in range(0, n, chunk)]
        done = 0
        next_log = 0.1
        ctx = mp.get_context("spawn")
        with ctx.Pool(workers, initializer=_init, initargs=(spec,)) as pool:
            for a, b, res in pool.imap_unordered(_work, ranges):
                for k in ("C", "T", "F", "n_placed", "n_eval"):
                    out[k][a:b] = res[k]
                if "k_mismatch_rays" in res:
                    bad.append(res["k_mismatch_rays"])
                done += b - a
                if log is not None and done >= next_log * n:
                    log(f"  oracle pool: {done}/{n} rays, {time.time() - t0:.1f} s")
                    next_log += 0.1
        out["seconds"] = time.time() - t0
        out["workers"] = workers
        if k_list is not None:
            out["k_mismatch_rays"] = np.sort(np.concatenate(bad)) if bad else np.zeros(0, np.int64)
        return out
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
