"""The persistent kernel's ticket protocol, modelled with host threads.

``tests/protocol/ticket_protocol.cpp`` plays every block of the persistent
batch kernel as a std::thread using the launcher's own schedule builder, and
checks that each tile runs once, after every tile of its scenario's previous
round, without deadlock.  It is built twice: plainly, and with
ThreadSanitizer (host code only), which reports any missing happens-before
edge between a tile's writes and the next round's reads as a data race.
"""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "protocol", "ticket_protocol.cpp")


def _build_and_run(tmp_path, extra, reps, env=None):
    exe = tmp_path / ("proto" + "_".join(x.strip("-=") for x in extra))
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-pthread", *extra, "-o", str(exe), SRC]
    subprocess.run(cmd, check=True)
    r = subprocess.run([str(exe), str(reps)], capture_output=True, text=True, timeout=600, env=env)
    return r


def test_ticket_protocol_plain(tmp_path):
    r = _build_and_run(tmp_path, [], 8)
    assert r.returncode == 0, r.stderr
    assert r.stdout.startswith("OK")


def test_ticket_protocol_under_thread_sanitizer(tmp_path):
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66")
    try:
        r = _build_and_run(tmp_path, ["-fsanitize=thread"], 2, env)
    except subprocess.CalledProcessError:
        pytest.skip("ThreadSanitizer is not available to g++ here")
    assert r.returncode == 0, r.stderr[-4000:]
    assert "WARNING: ThreadSanitizer" not in r.stderr
    assert r.stdout.startswith("OK")


def test_thread_sanitizer_catches_a_planted_missing_release(tmp_path):
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66")
    try:
        r = _build_and_run(tmp_path, ["-fsanitize=thread", "-DPLANT_MISSING_RELEASE"], 1, env)
    except subprocess.CalledProcessError:
        pytest.skip("ThreadSanitizer is not available to g++ here")
    assert r.returncode == 66 and "data race" in r.stderr
