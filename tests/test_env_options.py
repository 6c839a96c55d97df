"""Options from the environment (SS_<NAME> for every SS_OPT_<NAME>) and the
SS_LOG decision log, checked in child processes that load the library
(no GPU needed: options are host state)."""
import os
import subprocess
import sys

REPO = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys
sys.path.insert(0, {repo!r})
from paper_2112_03229_amd import binding as b
names = ["FORCE_ALGO", "BUCKET_BITS", "PLAN_ALGO", "CONVENTION", "PLAN_XCD", "PLAN_TILES"]
print(" ".join(str(b.get_option(getattr(b, "OPT_" + k))) for k in names))
"""


def run(env_extra):
    env = {k: v for k, v in os.environ.items() if not k.startswith("SS_")}
    env.update(env_extra)
    r = subprocess.run([sys.executable, "-c", CHILD.format(repo=REPO)], env=env,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    return [int(v) for v in r.stdout.split()], r.stderr


def test_defaults_without_environment():
    vals, err = run({})
    assert vals == [0, -1, 0, 0, 0, 0]
    assert "[ss]" not in err


def test_environment_sets_options():
    from paper_2112_03229_amd import binding as b
    vals, err = run({"SS_FORCE_ALGO": "exphash", "SS_BUCKET_BITS": "7", "SS_PLAN_ALGO": "ballot",
                     "SS_CONVENTION": "1", "SS_PLAN_XCD": "16", "SS_PLAN_TILES": "3"})
    assert vals == [b.ALGO_EXPHASH, 7, b.ALGO_BALLOT, 1, 16, 3]
    assert "[ss]" not in err  # applied silently without SS_LOG


def test_environment_numbers_and_log():
    vals, err = run({"SS_FORCE_ALGO": "1", "SS_LOG": "1"})
    assert vals[0] == 1
    assert "[ss] option SS_FORCE_ALGO = 1 (environment)" in err


def test_refused_values_are_reported_and_ignored():
    vals, err = run({"SS_BUCKET_BITS": "21", "SS_PLAN_XCD": "many", "SS_CONVENTION": "2",
                     "SS_PLAN_ALGO": "learned", "SS_LOG": "x", "SS_PLAN_TILES": "4"})
    assert vals == [0, -1, 0, 0, 0, 4]
    for name in ("SS_BUCKET_BITS=21", "SS_PLAN_XCD=many", "SS_CONVENTION=2",
                 "SS_PLAN_ALGO=learned", "SS_LOG=x"):
        assert f"[ss] ignoring {name}" in err, err
