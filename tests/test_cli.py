"""The command-line program: usage errors (CPU) and its byte stream against
the oracle (GPU). With seed 0 the stream is the paper's program output."""
import os
import subprocess

import numpy as np
import pytest

from paper_1609_01257_amd import build

CLI = build.CLI


def _run(*args, timeout=120):
    if not os.path.exists(CLI):
        pytest.fail("rngx_cli is not built (run __graft_entry__.build())")
    return subprocess.run([CLI, *map(str, args)], capture_output=True, timeout=timeout)


@pytest.mark.parametrize("args", [(), ("5",), ("0", "3"), ("5", "-1"), ("x", "3"),
                                  ("5", "3", "7"), ("-k", "0", "5", "3"), ("-s",),
                                  ("4294967296", "1"), ("-h", "0", "5", "3"),
                                  ("-k", "4294967295", "-h", "4294967295", "4294967295",
                                   "4294967295")])
def test_usage_errors(args):
    r = _run(*args)
    assert r.returncode == 2 and b"usage:" in r.stderr and r.stdout == b""


@pytest.mark.gpu
@pytest.mark.parametrize("args,seed,n,i,u32", [
    ((1000, 7), 0, 1000, 7, False),             # the paper's program, seed 0
    (("-k", 3, 777, 10), 0, 777, 10, False),    # 3 whole steps and a remainder of 1
    (("-s", "0x2a", "-u", "-h", 3, 4099, 5), 42, 4099, 5, True),
    ((65536, 0), 0, 65536, 0, False),           # zero iterations: no output
])
def test_stream_matches_oracle(oracle, args, seed, n, i, u32):
    r = _run(*args)
    assert r.returncode == 0, r.stderr.decode()
    exp = (oracle.generate_u32 if u32 else oracle.generate)(seed, n, i)
    assert r.stdout == exp.tobytes()


@pytest.mark.gpu
@pytest.mark.parametrize("u32", [False, True])
def test_scrambled_stream_matches_oracle(oracle, u32):
    args = ["-x", "-s", 5, "-k", 2, 3001, 7] + (["-u"] if u32 else [])
    r = _run(*args)
    assert r.returncode == 0, r.stderr.decode()
    exp = (oracle.generate_star_u32 if u32 else oracle.generate_star)(5, 3001, 7)
    assert r.stdout == exp.tobytes()
