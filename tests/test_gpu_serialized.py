"""The same outputs with and without the ROCm runtime serialising every
kernel and copy (AMD_SERIALIZE_KERNEL=3, AMD_SERIALIZE_COPY=3): no result
may depend on how the work of different streams interleaves."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

HELPER = os.path.join(os.path.dirname(os.path.abspath(__file__)), "helpers", "serialized_run.py")


def _child(extra_env):
    env = dict(os.environ)
    env.update(extra_env)
    r = subprocess.run([sys.executable, HELPER], capture_output=True, text=True, env=env,
                       timeout=110)
    assert r.returncode == 0, r.stderr[-2000:]
    return r.stdout.strip().splitlines()[-1]


@pytest.mark.timeout(300)   # two child processes, each importing torch
def test_serialized_runtime_gives_identical_outputs():
    plain = _child({})
    serial = _child({"AMD_SERIALIZE_KERNEL": "3", "AMD_SERIALIZE_COPY": "3"})
    assert len(plain) == 64 and plain == serial
