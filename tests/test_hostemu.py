"""CPU: the library's HIP sources built for the host (tests/hostemu) and run
under bounds checks: every array of block memory is index-checked (a trap on
any access outside it), every device buffer sits against an inaccessible page
(at its end, or at its start), block memory is filled with a poison pattern
before each block, and the threads of a block meet at real barriers.  Each
case also matches the oracle track by track.  This checks memory safety and
the block logic (pool refill, block stack, pending photons, deposit cache,
queue claims, claim order) of the same code the GPU runs; the GPU tests
remain the parity tests of the product."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, os.path.join(HERE, "hostemu"))

# (guard side, cases, blocks in concurrent processes)
RUNS = [
    ("end", ["tiny", "tiny_rot", "calorimeter", "pair_heavy", "barrel", "endcap", "multi"], False),
    ("start", ["pair_heavy", "barrel", "endcap"], False),
    ("end", ["calorimeter", "endcap", "multi"], True),
]
# configurations of the multi-geometry case (see run_cases.multi_case)
MULTI = {False: 3, True: 2}


@pytest.fixture(scope="module")
def emu_dir():
    import build_hostemu
    return build_hostemu.build()


def _start(emu_dir, guard, cases, fork):
    env = dict(os.environ, HOSTEMU_GUARD=guard, HOSTEMU_BARRIER_S="60")
    if fork:
        env.update(HOSTEMU_FORK="4", HOSTEMU_CUS="4")
    cmd = [sys.executable, "-u", os.path.join(HERE, "hostemu", "run_cases.py"), emu_dir, ",".join(cases)]
    if fork:
        cmd.append("fork")
    return subprocess.Popen(cmd, env=env, cwd=ROOT, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)


def test_transport_bounds_checked(emu_dir):
    """Every case and launch configuration; device buffers guarded at their
    end, then at their start; then blocks of one launch in concurrent
    processes that share the queue and the tallies, as blocks on the GPU do."""
    procs = [(run, _start(emu_dir, *run)) for run in RUNS]
    for (guard, cases, fork), p in procs:
        out, err = p.communicate(timeout=600)
        report = out + err[-3000:]
        assert p.returncode == 0, f"guard {guard}, fork {fork}: exit status {p.returncode}\n{report}"
        assert "BAD" not in out, report
        from run_cases import CONFIGS, FORK_CONFIGS
        single = [c for c in cases if c != "multi"]
        want = len(single) * len(FORK_CONFIGS if fork else CONFIGS) + (MULTI[fork] if "multi" in cases else 0)
        assert out.count("OK") == want, report
