"""Progress lines for long GPU tests: to stderr, and appended to the file named
by $HUSKY_PROGRESS_LOG when it is set."""

import os
import sys
import time

_T0 = time.time()


def say(*parts):
    msg = f"[{time.time() - _T0:7.1f}s] " + " ".join(str(p) for p in parts)
    print(msg, file=sys.stderr, flush=True)
    path = os.environ.get("HUSKY_PROGRESS_LOG")
    if path:
        with open(path, "a") as f:
            f.write(msg + "\n")
