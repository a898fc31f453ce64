"""CPU checks of the C ABI: the library loads, exports every function include/gmc.h declares,
and rejects bad arguments before touching a device."""
import ctypes
import os
import re
import subprocess
import sys

import numpy as np
import pytest

from paper_2512_13965_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include")))
           if f.endswith(".h")]


def _declared_functions():
    names = []
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                            text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "return")))


@pytest.fixture(scope="module")
def binding():
    from paper_2512_13965_amd import binding as b
    b.lib()
    return b


def test_header_compiles_as_c():
    for h in HEADERS:
        subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Werror", "-fsyntax-only", "-x", "c", h])


def test_every_declared_symbol_is_exported(binding):
    names = _declared_functions()
    assert "gmc_transmit" in names and "mc_transmit" in names
    out = subprocess.check_output(["nm", "-D", "--defined-only", binding.LIB_PATH], text=True)
    exported = set(l.split()[-1] for l in out.splitlines() if l.strip())
    missing = [n for n in names if n not in exported]
    assert not missing, missing


def test_host_checks(binding):
    from tests import abi_host_checks
    abi_host_checks.run(binding.lib())


def test_host_checks_under_address_and_undefined_behaviour_sanitizers():
    # the host code (blob parsing, argument checks) built with -fsanitize=address,undefined on the
    # host side only, exercised in a child process with the sanitizer runtime preloaded
    from paper_2512_13965_amd import _build
    lib = _build.ASAN_LIB if os.path.exists(_build.ASAN_LIB) else _build.build_asan()
    env = dict(os.environ, LD_PRELOAD=_build.asan_runtime(), ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-m", "tests.abi_host_checks", lib], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "host checks passed" in r.stdout, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
