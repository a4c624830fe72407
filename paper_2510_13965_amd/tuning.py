"""On-disk cache of the level autotuner's choices.

mhd_level_autotune times 27 launch shapes on the level itself (seconds on a
large level).  The choice depends on the device, the library version, whether
radiation is evolved and the set of box shapes, not on the field values, so it
is stored under a key made of exactly those and reused by later levels of the
same shape.  The cache is one JSON object {key: tuning} written atomically
(temporary file + rename); an unreadable file counts as empty.
"""
import hashlib
import json
import os

TUNING_KEYS = ("strip", "block_threads", "grid_per_cu")


def cache_key(box_dims, m1, device, abi):
    """Key of a level: box_dims is an iterable of (nx, ny, nz); their order does
    not matter (the tile layout sorts nothing, but the timed work is the same
    multiset of boxes)."""
    dims = sorted(tuple(int(v) for v in d) for d in box_dims)
    blob = json.dumps({"abi": int(abi), "device": str(device), "m1": bool(m1), "boxes": dims}, sort_keys=True)
    return hashlib.sha256(blob.encode()).hexdigest()[:32]


class TuningCache:
    def __init__(self, path):
        self.path = os.fspath(path)

    def _load(self):
        try:
            with open(self.path) as fh:
                data = json.load(fh)
        except (OSError, ValueError):
            return {}
        return data if isinstance(data, dict) else {}

    def get(self, key):
        t = self._load().get(key)
        if not isinstance(t, dict) or any(not isinstance(t.get(k), int) for k in TUNING_KEYS):
            return None
        return {k: t[k] for k in TUNING_KEYS}

    def put(self, key, tuning):
        data = self._load()
        data[key] = {k: int(tuning[k]) for k in TUNING_KEYS}
        d = os.path.dirname(os.path.abspath(self.path))
        os.makedirs(d, exist_ok=True)
        tmp = "%s.%d.tmp" % (self.path, os.getpid())
        with open(tmp, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
        os.replace(tmp, self.path)
