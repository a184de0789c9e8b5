"""Oracle builds with a planted mistake, for tests that show a pin catches it.

A variant is the oracle's own source with one text replacement applied (the replaced text
must occur exactly once), compiled with the oracle's flags into a temporary directory and
loaded with the oracle's typed signatures.  Runs on the CPU only.
"""
import hashlib
import os
import shutil
import subprocess
import tempfile

import oracle
from oracle.build import HERE, SOURCES

_cache = {}


def build_variant(file: str, old: str, new: str):
    """Library handle of the oracle with `old` replaced by `new` in oracle/<file>."""
    key = hashlib.sha1(f"{file}\0{old}\0{new}".encode()).hexdigest()[:16]
    if key in _cache:
        return _cache[key]
    d = tempfile.mkdtemp(prefix=f"orc_variant_{key}_")
    for name in SOURCES + ["oracle.h"]:
        shutil.copy(os.path.join(HERE, name), os.path.join(d, name))
    path = os.path.join(d, file)
    src = open(path).read()
    assert src.count(old) == 1, f"planted text must occur once in {file}: {old!r}"
    open(path, "w").write(src.replace(old, new))
    lib = os.path.join(d, "liboracle_variant.so")
    subprocess.run(["g++", "-std=c++17", "-O1", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-shared",
                    "-fPIC", "-o", lib, *[os.path.join(d, s) for s in SOURCES]], check=True)
    _cache[key] = oracle.load(lib)
    return _cache[key]
