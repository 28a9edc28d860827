"""Progress lines of the GPU tests. They are written past pytest's output capture, so that a long test (a full-size
comparison with the oracle runs for minutes) keeps printing under -q as well as under -s; outside pytest they are
plain prints."""
import sys

_config = None  # set by conftest.pytest_configure


def say(*a):
    msg = " ".join(str(x) for x in a)
    capman = _config.pluginmanager.getplugin("capturemanager") if _config is not None else None
    if capman is None:
        print(msg, flush=True)
        return
    with capman.global_and_fixture_disabled():
        sys.stdout.write(msg + "\n")
        sys.stdout.flush()
