"""Cache of the library's measured launch choices (selinv_tune).

The tuning table of a handle (tile edge per launch class, fused or per-phase
launches for the levels of small supernodes, stored G or G read from its
sources per level, sweep form) depends on the
plan's shape, the precision, the device and the library build.  ``tuned``
looks the table up in a JSON file under that key and installs it, or runs
the tuner and stores the result.
"""
from __future__ import annotations

import hashlib
import json
import os

from . import selinv

DEFAULT_CACHE = os.path.join(os.environ.get("XDG_CACHE_HOME", os.path.expanduser("~/.cache")),
                             "paper_1708_04539_amd", "tuning.json")


def _library_digest() -> str:
    h = hashlib.sha256()
    with open(selinv.LIB_PATH, "rb") as f:
        for chunk in iter(lambda: f.read(1 << 20), b""):
            h.update(chunk)
    return h.hexdigest()[:16]


def plan_key(s: "selinv.SelInv", precision: str, device: str = "") -> str:
    """Key of one (plan shape, precision, device, library build)."""
    st = s.structure()
    h = hashlib.sha256()
    for k in ("xsup", "rl_ptr", "ru_ptr", "level"):
        h.update(st[k].tobytes())
    return f"{device}|{precision}|{s.info['symbolic']}|{h.hexdigest()[:24]}|{_library_digest()}"


def _device_name() -> str:
    try:
        import torch
        return torch.cuda.get_device_name(0) if torch.cuda.is_available() else ""
    except Exception:  # pragma: no cover - torch is part of the image
        return ""


def tuned(s: "selinv.SelInv", precision: str = "fp64", cache_path: str | None = DEFAULT_CACHE, reps: int = 5,
          stream=None) -> dict:
    """Install the cached tuning table of ``s`` for ``precision``, or tune and
    cache it.  Returns {"table", "cached", "ms_policy", "ms_tuned"}."""
    key = plan_key(s, precision, _device_name())
    cache = {}
    if cache_path and os.path.exists(cache_path):
        try:
            with open(cache_path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    ent = cache.get(key)
    if ent is not None:
        s.set_tuning(ent["table"], precision)
        return {"table": ent["table"], "cached": True, "ms_policy": ent.get("ms_policy"),
                "ms_tuned": ent.get("ms_tuned")}
    ms_pol, ms_tun = s.tune(precision, reps, stream)
    table = s.get_tuning(precision)
    if cache_path:
        cache[key] = {"table": table, "ms_policy": ms_pol, "ms_tuned": ms_tun}
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f)
        os.replace(tmp, cache_path)
    return {"table": table, "cached": False, "ms_policy": ms_pol, "ms_tuned": ms_tun}


def describe(table: list) -> dict:
    """Readable summary of a tuning table (side_inversion_chunk: the number of
    workgroups of the side stream's inversion launches, 0 for one per item)."""
    if not table:
        return {"tuned": False}
    L = table[1]
    hd = {4: 8, 3: 8, 2: 7}.get(table[0], 6)
    pl = 4 if table[0] == 4 else 3
    per = [table[hd + pl * d: hd + pl + pl * d] for d in range(L)]
    return {"tuned": True, "sweep": {0: "handle", 1: "levels", 2: "persistent"}[table[2]],
            "prologue_tiles": {"tri": table[3], "norm": table[4], "diag_init": table[5]},
            "prologue_side_stream": not (hd >= 7 and table[6] == 1),
            "prologue_part_per_level": hd >= 7 and table[6] == 2,
            "side_inversion_chunk": table[7] if hd == 8 else 0,
            "steps35_tiles": [p[0] for p in per], "step4_tiles": [p[1] for p in per],
            "small_per_phase_levels": [d for d, p in enumerate(per) if p[2]],
            "gather_in_products_levels": [d for d, p in enumerate(per) if pl == 4 and p[3]]}
