"""The oracle's pins catch plausible mistakes (CPU only).

Each case plants one mistake in a copy of the oracle (oracle.c or the
network oracle mlp.py) in a temporary directory, builds that copy, and runs
the oracle pin tests (tests/test_oracle_*.py) against it in a subprocess;
some pin must fail.  The mistakes are the kind a transcription of the paper
would make: a rounding or a sign in the colour transform (Sec. 4), a field
width or digit order in BISE (Sec. 3.3), the zigzag and the quantiser
(Sec. 3.2), the cluster filter's weights and rounding (eq. 2), the rank of a
node in its group (Sec. 3.4), a level dropped from the gather (Alg. 2), the
image padding, the block-energy threshold (Sec. 3.2), the tree's indexing
(Sec. 3.1), the render's fractions, pixel centres and focal shift
(Sec. 3.6), progressive decompression's stopping level, the PSNR weights
(eqs. 4-5), the clamp, and the network oracle's ReLU, bias, back-propagation
and Adam step.
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# (name, file, text in the oracle, replacement)
MUTATIONS = [
    ("ycocg_forward_rounding", "oracle.c", "int32_t t = b + (int32_t)floor_div(o, 2);",
     "int32_t t = b + (int32_t)floor_div(o + 1, 2);"),
    ("ycocg_inverse_sign", "oracle.c", "*b = t - (int32_t)floor_div(co, 2);", "*b = t + (int32_t)floor_div(co, 2);"),
    ("trit_field_width", "oracle.c", "if (kind == KIND_TRIT) return (int)ceil_div(8 * k, 5);",
     "if (kind == KIND_TRIT) return (int)ceil_div(8 * k, 4);"),
    ("digit_order", "oracle.c", "digit[i + r] = number % (uint32_t)rdx;", "digit[i + k - 1 - r] = number % (uint32_t)rdx;"),
    ("zigzag_negative", "oracle.c", "return v >= 0 ? 2 * v : -2 * v - 1;", "return v >= 0 ? 2 * v : -2 * v + 1;"),
    ("unzigzag_odd", "oracle.c", "-(z + 1) / 2;", "-(z - 1) / 2;"),
    ("filter_weights_transposed", "oracle.c", "weights[nm] = binom(c - 1, cx) * binom(c - 1, cy);",
     "weights[nm] = binom(c - 1, cx) * binom(c - 1, cx);"),
    ("filter_rounding", "oracle.c", "dst[i] = (int32_t)floor_div(acc + wt / 2, wt);",
     "dst[i] = (int32_t)floor_div(acc, wt);"),
    ("rank_off_by_one", "oracle.c", "if (get_bit(gw, k)) { if (k < s) rank++; np++; }",
     "if (get_bit(gw, k)) { if (k <= s) rank++; np++; }"),
    # the random-access reader's payload start (the encoder and the whole-field
    # reader keep theirs)
    ("code_section_length", "oracle.c",
     "  int64_t code_bit = 32LL * nbw;\n  int64_t pay_bit = 32LL * (nbw + ceil_div(5 * np, 32));",
     "  int64_t code_bit = 32LL * nbw;\n  int64_t pay_bit = 32LL * (nbw + ceil_div(5 * np + 5, 32));"),
    ("gather_drops_level0", "oracle.c", "for (int l = L - 2; l >= 0; l--) {               /* GetParentIndices",
     "for (int l = L - 2; l >= 1; l--) {               /* GetParentIndices"),
    ("padding_not_replicated", "oracle.c", "int sx = x < p->width ? x : p->width - 1;", "int sx = x < p->width ? x : 0;"),
    ("energy_threshold_inclusive", "oracle.c", "int present = energy > p.blk_threshold;",
     "int present = energy >= p.blk_threshold;"),
    ("ancestor_transposed", "oracle.c", "  return y * t->lu[l] + x;\n}", "  return x * t->lv[l] + y;\n}"),
    ("render_v_fraction", "oracle.c", "lv[a] = lerpf(lt[0], lt[1], fv);", "lv[a] = lerpf(lt[0], lt[1], fu);"),
    ("render_pixel_centre", "oracle.c", "float sx = s + ((float)X + 0.5f) * sxs - 0.5f;", "float sx = s + (float)X * sxs;"),
    ("render_focal_sign", "oracle.c", "float dx = d == 0.0f ? 0.0f : d * ((float)iu[a] - uc);",
     "float dx = d == 0.0f ? 0.0f : d * (uc - (float)iu[a]);"),
    ("progressive_stop", "oracle.c", "for (int l = L - 2; l >= level; l--) {", "for (int l = L - 2; l > level; l--) {"),
    ("psnr_weights", "oracle.c", "total += (6.0 * ps[0] + ps[1] + ps[2]) / 8.0;", "total += (ps[0] + ps[1] + ps[2]) / 3.0;"),
    ("clamp_255", "oracle.c", "return v < 0 ? 0 : (v > 255 ? 255 : v);", "return v < 0 ? 0 : (v > 254 ? 254 : v);"),
    ("mlp_relu", "mlp.py", "h1 = np.maximum(x @ p[\"W1\"].T + p[\"b1\"], 0)", "h1 = x @ p[\"W1\"].T + p[\"b1\"]"),
    ("mlp_missing_bias", "mlp.py", "h2 = np.maximum(h1 @ p[\"W2\"].T + p[\"b2\"], 0)", "h2 = np.maximum(h1 @ p[\"W2\"].T, 0)"),
    ("quantiser_truncates", "oracle.c", "int32_t mag = (iabs32(r) + (1 << (q - 1))) >> q;", "int32_t mag = iabs32(r) >> q;"),
    ("adam_no_bias_correction", "mlp.py", "mh = m / (1 - beta1 ** step)", "mh = m"),
    ("backprop_relu_mask", "mlp.py", "dh1 = (dh2 @ p[\"W2\"]) * (h1 > 0)", "dh1 = dh2 @ p[\"W2\"]"),
]

PIN_TESTS = ["test_oracle_bise.py", "test_oracle_codec.py", "test_oracle_colour.py", "test_oracle_control.py",
             "test_oracle_progressive.py", "test_oracle_render.py", "test_oracle_tree.py"]


def _run_mutant(tmp, name, fname, old, new):
    """Builds the mutated oracle under tmp/name/oracle and runs the pins on it;
    returns (name, caught, detail)."""
    base = os.path.join(tmp, name)
    pkg = os.path.join(base, "oracle")
    shutil.copytree(os.path.join(ROOT, "oracle"), pkg,
                    ignore=shutil.ignore_patterns("*.so", "*.so.tmp", "__pycache__"))
    path = os.path.join(pkg, fname)
    with open(path) as fh:
        src = fh.read()
    if src.count(old) != 1:
        return name, False, f"the text to mutate occurs {src.count(old)} times in {fname}"
    with open(path, "w") as fh:
        fh.write(src.replace(old, new))
    b = subprocess.run([sys.executable, os.path.join(pkg, "build.py")], capture_output=True, text=True, timeout=300)
    if b.returncode:
        return name, True, "the mutant does not build"
    env = dict(os.environ, PYTHONPATH=os.pathsep.join([base, ROOT]), OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu", "-p", "no:cacheprovider",
                        *[os.path.join(ROOT, "tests", t) for t in PIN_TESTS]],
                       cwd=base, env=env, capture_output=True, text=True, timeout=600)
    # the pins must have run against the mutant: the import resolved to the copy
    return name, r.returncode != 0, (r.stdout + r.stderr)[-400:]


def test_mutant_import_resolves_to_the_copy(tmp_path):
    # the subprocess set-up puts the copied package ahead of the repository's
    pkg = tmp_path / "oracle"
    shutil.copytree(os.path.join(ROOT, "oracle"), pkg, ignore=shutil.ignore_patterns("*.so", "__pycache__"))
    env = dict(os.environ, PYTHONPATH=os.pathsep.join([str(tmp_path), ROOT]))
    out = subprocess.run([sys.executable, "-c", "import oracle; print(oracle.__file__)"], cwd=str(tmp_path),
                         env=env, capture_output=True, text=True, check=True).stdout.strip()
    assert out.startswith(str(tmp_path))


@pytest.mark.slow
def test_every_planted_mistake_is_caught(tmp_path):
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        results = list(ex.map(lambda m: _run_mutant(str(tmp_path), *m), MUTATIONS))
    missed = [(n, d) for n, caught, d in results if not caught]
    assert not missed, "mistakes the pins do not catch:\n" + "\n".join(f"{n}: {d}" for n, d in missed)
