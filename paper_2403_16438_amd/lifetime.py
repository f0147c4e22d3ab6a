"""Orderly release of the library's native objects.

Sessions hold HIP events, batch objects a captured graph, a stream, an event
and pinned host memory; networks and motion correctors hold host tables
bound to device memory. Each wrapper releases its object in close(). At
interpreter exit, finalizers run in no defined order and possibly after the
HIP runtime has started to tear itself down, so here:

* every wrapper registers itself with track() once its handle exists;
* shutdown() waits for the device, then closes every live wrapper, newest
  first; it runs by itself from an atexit hook registered when this package
  is imported (after torch, so it runs before torch's own exit hooks), and
  may be called earlier by a program that wants the release to happen at a
  point of its choosing; it is idempotent;
* a finalizer (__del__) releases nothing once shutdown() has started or the
  interpreter is finalizing (see released_by_finalizer()).
"""
from __future__ import annotations

import atexit
import itertools
import sys
import threading
import weakref

_lock = threading.Lock()
_live: "dict[int, weakref.ref]" = {}
_ids = itertools.count()
_closing = False


def track(obj) -> None:
    """Register a wrapper with a close() method for release at shutdown."""
    with _lock:
        key = next(_ids)
        _live[key] = weakref.ref(obj, lambda _r, k=key: _live.pop(k, None))


def released_by_finalizer() -> bool:
    """True while a finalizer may still release native objects."""
    return not _closing and not sys.is_finalizing()


def shutdown() -> None:
    """Wait for the device, then close every live wrapper, newest first."""
    global _closing
    with _lock:
        if _closing:
            return
        _closing = True
        refs = [r for _, r in sorted(_live.items(), reverse=True)]
        _live.clear()
    try:
        import torch
        if torch.cuda.is_initialized():
            torch.cuda.synchronize()
    except Exception:
        pass
    for r in refs:
        obj = r()
        if obj is not None:
            try:
                obj.close()
            except Exception:
                pass


atexit.register(shutdown)
