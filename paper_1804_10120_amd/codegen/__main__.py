"""Regenerates the generated kernels, header and manifest from the registry:

    python -m paper_1804_10120_amd.codegen [--check]

--check exits with status 1 if the committed files differ from what the
registry generates (without writing anything).
"""
import json
import os
import sys

from .emit import generate
from .registry import programs

PKG = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROOT = os.path.dirname(PKG)
FILES = {
    "source": os.path.join(PKG, "csrc", "generated", "tlg_kernels.hip"),
    "header": os.path.join(ROOT, "include", "tl_generated.h"),
    "manifest": os.path.join(PKG, "generated.json"),
}


def contents():
    src, hdr, man = generate(programs())
    return {"source": src, "header": hdr, "manifest": json.dumps(man, indent=1) + "\n"}


def main(argv):
    new = contents()
    if "--check" in argv:
        stale = [k for k, path in FILES.items()
                 if not os.path.exists(path) or open(path).read() != new[k]]
        if stale:
            print("stale generated files:", ", ".join(FILES[k] for k in stale))
            return 1
        return 0
    for k, path in FILES.items():
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path, "w") as f:
            f.write(new[k])
        print("wrote", path)
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
