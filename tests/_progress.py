"""Progress lines from long GPU tests that reach the terminal even while
pytest captures the test's output (-q without -s), so a runner watching the
output sees a long test advance."""
import sys

_capman = None  # pytest's capture manager, registered by conftest.py


def register(capman):
    global _capman
    _capman = capman


def say(*a):
    if _capman is not None:
        with _capman.global_and_fixture_disabled():
            print(*a, flush=True)
    else:
        print(*a, flush=True)
    sys.stdout.flush()
