"""Launch-option cache for the connectivity kernels.

`tuned.json` maps a key (form, graph class, log2 of n rounded) to the
cc_set_option values the autotuner measured fastest for it; lookups fall back
to the nearest size of the same form and class, then to the library defaults.
No option changes any result, only speed.
"""
from __future__ import annotations

import json
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuned.json")
DEFAULTS = {"update_mode": 0, "block": 256, "items": 0, "query_halving": 1, "compress_every": 0,
            "hook": 0, "grid_cap": 4096, "compress_linked": 1, "filter": 0, "query_items": 0, "split_below": 0}


def _load():
    if not os.path.exists(CACHE):
        return {}
    with open(CACHE) as f:
        return json.load(f)


def key(form: str, workload: str, n: int) -> str:
    return "%s/%s/%d" % (form, workload, int(round(math.log2(max(1, n)))))


def lookup(form: str, workload: str, n: int) -> dict:
    tab = _load()
    k = key(form, workload, n)
    if k in tab:
        return dict(tab[k])
    best, bd = None, None
    lg = round(math.log2(max(1, n)))
    for kk, v in tab.items():
        f, w, s = kk.split("/")
        if f == form and w == workload:
            d = abs(int(s) - lg)
            if bd is None or d < bd:
                best, bd = v, d
    return dict(best) if best else {}


def plain_options(n: int, workload: str = "rmat") -> dict:
    o = dict(DEFAULTS)
    o.update(lookup("plain", workload, n))
    return o


def store(form: str, workload: str, n: int, options: dict, meta: dict | None = None):
    tab = _load()
    e = dict(options)
    tab[key(form, workload, n)] = e
    with open(CACHE, "w") as f:
        json.dump(tab, f, indent=1, sort_keys=True)
