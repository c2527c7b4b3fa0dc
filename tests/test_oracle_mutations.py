"""The oracle's pins catch plausible mistakes.

Each case plants one plausible mistake in a copy of the oracle's C source (in a
temporary directory, on the CPU), rebuilds it, and runs the pin suite against
the copy: the suite must fail.  The committed oracle itself is never modified.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTATIONS = [
    ("weight constant off by 1e-7", "c = c * (2.0 * t);", "c = c * (2.0 * t) * 1.0000001;"),
    ("boosted energy sign", "v[0] = gamma * e + ep;", "v[0] = gamma * e - ep;"),
    ("boost 1/(gamma-1)", "const double f = ep / (gamma + 1.0) + e;", "const double f = ep / (gamma - 1.0) + e;"),
    ("sin/cos swapped", "nhat[0] = st * cos(phi);", "nhat[0] = st * sin(phi);"),
    ("cos(theta) sign", "const double ct = 2.0 * u - 1.0;", "const double ct = 1.0 - 2.0 * u;"),
    ("mass uniforms not sorted", "sort_ascending(&r[1], n - 2);", ""),
    ("theta/phi uniforms swapped", "direction(u[n - 2 + 2 * i], u[n - 1 + 2 * i], nhat);",
     "direction(u[n - 1 + 2 * i], u[n - 2 + 2 * i], nhat);"),
    ("wrong uniform bits", "uint64_t x = bits >> 12;", "uint64_t x = (bits >> 11) & ((1ull << 52) - 1);"),
    ("factorial off by one", "for (int i = 2; i <= n - 2; ++i) fact", "for (int i = 2; i <= n - 3; ++i) fact"),
    ("Philox key word", "uint32_t y2 = hi0 ^ x3 ^ k1;", "uint32_t y2 = hi0 ^ x3 ^ k0;"),
    ("subsystem not back to back", "rest[k + 1] = -(p[i] * nhat[k]);", "rest[k + 1] = (p[i] * nhat[k]);"),
    ("parent gamma off by 1e-6", "const double gamma = parent4[0] / parent_mass;",
     "const double gamma = parent4[0] / parent_mass * 1.000001;"),
    ("variance scaled", "nsum_add(&s2, d * d);", "nsum_add(&s2, d * d * 1.0000001);"),
    ("emitted daughter not boosted", "boost(dau, eta, gamma);", ""),
    ("remaining subsystem not boosted", "boost(rest, eta, gamma);", ""),
    ("subsystem boost reversed", "eta[k] = sub[k + 1] / sigma[i + 1];", "eta[k] = -sub[k + 1] / sigma[i + 1];"),
    ("subsystem gamma from the inner mass", "const double gamma = sub[0] / sigma[i + 1];",
     "const double gamma = sub[0] / sigma[i];"),
    ("accept uniform from the event's own last call", "(uint32_t)oracle_calls_per_event(n), stream_id };",
     "(uint32_t)(oracle_calls_per_event(n) - 1), stream_id };"),
    ("accept test inverted", "if (v * w_max < w) {", "if (v * w_max > w) {"),
    ("sample maximum not taken", "if (w > w_max) w_max = w;", "if (w > w_max) w_max = w * 0.5;"),
    ("kept events stored at the trial index", "out[(uint64_t)(4 * d + mu) * ld + kept] = p4[d][mu];",
     "out[(uint64_t)(4 * d + mu) * ld + e] = p4[d][mu];"),
    ("Breit-Wigner denominator sign", "const double d = mass[k] * mass[k] - s;",
     "const double d = mass[k] * mass[k] + s;"),
    ("pair momentum differenced", "x = a[1] + b[1], y = a[2] + b[2]", "x = a[1] - b[1], y = a[2] + b[2]"),
    ("Breit-Wigner width term", "const double mg = mass[k] * width[k];", "const double mg = width[k];"),
    ("model unweighting on the weight alone", "return w * model_intensity(p4, model->n_bw",
     "return w + 0.0 * model_intensity(p4, model->n_bw"),
    ("VEGAS Jacobian without the bin count",
     "val = val * gauss_factor(x, mu[d], sig[d]) * ((double)bins * width * (hi[d] - lo[d]));",
     "val = val * gauss_factor(x, mu[d], sig[d]) * (width * (hi[d] - lo[d]));"),
    ("VEGAS point inside the bin", "const double y = g[b] + (z - (double)b) * width;",
     "const double y = g[b] + u * width;"),
    ("VEGAS damping exponent sign", "r[k] = R > 1.0 ? pow((1.0 - 1.0 / R) / log(R), alpha) : 1.0;",
     "r[k] = R > 1.0 ? pow((1.0 - 1.0 / R) / log(R), -alpha) : 1.0;"),
    ("VEGAS histogram not smoothed", "tot += sm[k];", "sm[k] = h[k];\n            tot += sm[k];"),
    ("VEGAS end-bin smoothing over three", "if (k == 0) sm[k] = (h[0] + h[1]) / 2.0;",
     "if (k == 0) sm[k] = (h[0] + h[1]) / 3.0;"),
    ("VEGAS new edge mirrored in the old bin", "edges[e] = g[k] + frac * (g[k + 1] - g[k]);",
     "edges[e] = g[k] + (1.0 - frac) * (g[k + 1] - g[k]);"),
]


# Each planted mistake runs the pins of the part it lives in (a -k expression
# over the pin names), so the suite stays short; every pin still runs against
# the mistakes of its own part.
PIN_GROUPS = {
    "events": "not model and not vegas and not plain_mc and not unweight and not accept and not kept",
    "unweighting": "unweight or accept or kept",
    "model": "model",
    "vegas": "vegas or plain_mc",
}


def _group(name: str) -> str:
    if name.startswith("VEGAS"):
        return "vegas"
    if "Breit-Wigner" in name or "pair momentum" in name or name.startswith("model"):
        return "model"
    if name.startswith(("accept", "sample maximum", "kept events")):
        return "unweighting"
    return "events"


@pytest.mark.slow
@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_planted_mistake(tmp_path, name, old, new):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    work = tmp_path / "w"
    shutil.copytree(os.path.join(ROOT, "oracle"), work / "oracle",
                    ignore=shutil.ignore_patterns("*.so", "__pycache__"))
    src = work / "oracle" / "phsp_oracle.c"
    text = src.read_text()
    assert old in text, f"mutation site not found: {old}"
    src.write_text(text.replace(old, new, 1))
    tests = work / "tests"
    tests.mkdir()
    for f in ("conftest.py", "volumes.py", "test_oracle_pins.py"):
        shutil.copy(os.path.join(ROOT, "tests", f), tests / f)
    shutil.copytree(os.path.join(ROOT, "tests", "kat"), tests / "kat")
    env = dict(os.environ, PYTHONPATH=str(work))
    subprocess.run([sys.executable, "-c", "import oracle; oracle.build()"], cwd=work, env=env, check=True)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-k", PIN_GROUPS[_group(name)], str(tests / "test_oracle_pins.py")], cwd=work, env=env,
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 1, f"planted mistake '{name}' passed every {_group(name)} pin:\n{r.stdout[-2000:]}"
