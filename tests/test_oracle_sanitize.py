"""The oracle under the address and undefined-behaviour sanitizers (CPU).

``oracle/sanitize_check.c`` includes the oracle's C source into one program
and drives every entry point on small seeded 2D and 3D cases (SDSD and SDMD
steps with and without the current filter, both deposition modes, the
diagnostics, binning, the split form, interpolation and Boris), with checks
that the two decompositions agree.  Built with gcc's
``-fsanitize=address,undefined`` and no recovery, any out-of-bounds access,
leak or undefined operation ends the run with a report; the test needs exit
status 0, "ok" and no sanitizer output.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "sanitize_check.c")
FLAGS = ["-O1", "-g", "-std=c99", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
         "-fno-omit-frame-pointer"]


def _build(tmp_path, src_text=None):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not found")
    exe = str(tmp_path / "sanitize_check")
    src = SRC
    if src_text is not None:
        src = str(tmp_path / "probe.c")
        with open(src, "w") as f:
            f.write(src_text)
    r = subprocess.run([gcc, *FLAGS, "-I", os.path.join(ROOT, "oracle"), src, "-lm", "-o", exe],
                       capture_output=True, text=True)
    if r.returncode != 0 and "asan" in (r.stderr + r.stdout).lower():
        pytest.skip("gcc has no sanitizer runtime here: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr
    return exe


def _run(exe):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    return subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)


def test_oracle_clean_under_asan_ubsan(tmp_path):
    r = _run(_build(tmp_path))
    assert r.returncode == 0, r.stderr[-3000:]
    assert r.stdout.strip() == "ok"
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]


def test_sanitizers_are_active(tmp_path):
    """The same build flags do catch a planted overflow in the oracle's own
    code (a copy of its source with one array read past its end)."""
    src = open(os.path.join(ROOT, "oracle", "pic_oracle.c")).read()
    planted = src + """
int planted_main(void);
int main(void) { return planted_main(); }
int planted_main(void)
{
    double *a = (double *)malloc(sizeof(double) * 4);
    for (int i = 0; i < 4; ++i) a[i] = i;
    volatile double s = 0.0;
    for (int i = 0; i <= 4; ++i) s += a[i];   /* reads a[4] */
    free(a);
    return (int)s;
}
"""
    r = _run(_build(tmp_path, planted))
    assert r.returncode != 0
    # whichever sanitizer reports first: ASan's overflow or UBSan's bad load
    assert "heap-buffer-overflow" in r.stderr or "runtime error: load of address" in r.stderr, r.stderr[-2000:]
