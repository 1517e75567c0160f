"""Run every pin of the oracle against one build of it (argument: the library path).

Used by tests/test_sanitizers.py with a build instrumented by AddressSanitizer and
UndefinedBehaviorSanitizer, in a process that preloads their runtimes: any invalid
access or undefined operation in oracle.c aborts the run.  Prints one line per pin."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

import oracle as O  # noqa: E402
import test_oracle_pins as pins  # noqa: E402

orc = O.Oracle(sys.argv[1])
failed = 0
for check in pins.CHECKS:
    msg = check(orc)
    print(f"{check.__name__}: {'ok' if msg is None else msg}", flush=True)
    failed += msg is not None
# the threaded paths (rows and inner products above 32768 entries) on two threads
orc.set_threads(2)
msg = pins.check_p16b(orc)
print(f"check_p16b (2 threads): {'ok' if msg is None else msg}", flush=True)
failed += msg is not None
sys.exit(1 if failed else 0)
