"""Content hash of the library's sources (csrc/ and include/eap.h).

The build embeds it in libeap.so (eap_source_hash()), and the binding refuses
a library whose hash differs from the sources next to it, so a stale build is
never tested or benchmarked silently.  Content, not file times: a copy of the
tree keeps the same hash.
"""
import hashlib
import os

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
HEADER = os.path.join(ROOT, "include", "eap.h")


def source_files():
    files = [os.path.join(CSRC, f) for f in sorted(os.listdir(CSRC)) if f.endswith((".hip", ".h", ".cpp"))]
    return files + [HEADER]


def source_hash() -> str:
    h = hashlib.sha256()
    for f in source_files():
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]
