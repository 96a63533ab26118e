"""Metrics as JSON lines: one object per event (a step's moments and time, a
request's completion, a run summary), each with its kind and a wall-clock
stamp, appended to a file and flushed line by line so that a reader (or a
crashed run) sees every completed event."""
from __future__ import annotations

import json
import math
import time


def _plain(v):
    if hasattr(v, "item") and getattr(v, "ndim", 1) == 0:
        v = v.item()
    if isinstance(v, float) and not math.isfinite(v):
        return str(v)
    if isinstance(v, dict):
        return {str(k): _plain(x) for k, x in v.items()}
    if isinstance(v, (list, tuple)):
        return [_plain(x) for x in v]
    return v


class MetricsLog:
    """Append-only JSONL writer; usable as a context manager."""

    def __init__(self, path: str):
        self.path = path
        self._fh = open(path, "a", buffering=1)

    def write(self, kind: str, **fields) -> None:
        rec = {"kind": kind, "wall": time.time()}
        rec.update({k: _plain(v) for k, v in fields.items()})
        self._fh.write(json.dumps(rec) + "\n")

    def close(self) -> None:
        if self._fh:
            self._fh.close()
            self._fh = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def read(path: str) -> list:
    with open(path) as fh:
        return [json.loads(line) for line in fh if line.strip()]
