"""Observed errors of the GPU parity tests.

When the environment variable SU2_ERROR_LOG names a file, every comparison a
parity test makes appends one JSON line to it: the test, what was compared
(configuration, direction, precision), the normwise relative error and the
worst element relative to the largest reference element.  The committed
precision summary is made from such a log; without the variable nothing is
written.
"""
import json
import os


def record(what, rel, worst, **extra):
    path = os.environ.get("SU2_ERROR_LOG")
    if not path:
        return
    entry = {"test": os.environ.get("PYTEST_CURRENT_TEST", "").split(" ")[0], "what": what,
             "rel": float(rel), "worst": float(worst)}
    entry.update(extra)
    with open(path, "a") as fh:
        fh.write(json.dumps(entry) + "\n")
