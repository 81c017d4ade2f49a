"""Mutation checks of the oracle's pins (CPU only).

Each case plants one plausible mistake in a temporary copy of a piece of the
oracle -- an edit of its C source compiled with gcc into a separate library,
or an edit of one of its Python functions executed in a copy of its module's
namespace -- and requires that at least one pin fails under it (a dropped
term or factor, a wrong sign, index, operand or constant).  The pins are the
tests of tests/test_oracle_*.py, each file loaded afresh for every case so
that it binds the mutated functions.  The unmutated oracle passes them all.
The committed oracle is never modified: a mutated piece replaces the original
(and every alias of it in the oracle package) only for one case.
"""
import ctypes
import importlib.util
import inspect
import itertools
import os
import subprocess
import tempfile
import textwrap

import pytest

import oracle
from oracle import dgl, functional, mlp, slq

HERE = os.path.dirname(os.path.abspath(__file__))
MODULES = (oracle, slq, dgl, functional, mlp)
CORE = ("test_oracle_pins.py",)


def _load_pins(filename):
    path = os.path.join(HERE, filename)
    spec = importlib.util.spec_from_file_location("pins_" + filename[:-3], path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _pin_calls(mod):
    """Every test function of a pin module, with its parametrize cases expanded."""
    calls = []
    for name, fn in sorted(vars(mod).items()):
        if not (name.startswith("test_") and inspect.isfunction(fn)):
            continue
        combos = [{}]
        for mark in getattr(fn, "pytestmark", []):
            if mark.name != "parametrize":
                continue
            argnames = mark.args[0]
            names = [a.strip() for a in argnames.split(",")] if isinstance(argnames, str) else list(argnames)
            values = [v if len(names) > 1 else (v,) for v in mark.args[1]]
            combos = [{**c, **dict(zip(names, v))} for c, v in itertools.product(combos, values)]
        for kw in combos:
            calls.append((f"{name}{kw if kw else ''}", lambda fn=fn, kw=kw: fn(**kw)))
    return calls


def _failing_pins(pin_files):
    failed = []
    for filename in pin_files:
        for name, call in _pin_calls(_load_pins(filename)):
            try:
                call()
            except Exception:  # an assertion, or the oracle failing outright
                failed.append(f"{filename}::{name}")
    return failed


# ---------------------------------------------------------------- C source
C_SRC = os.path.join(os.path.dirname(oracle.__file__), "kpm_oracle.c")
C_MUTATIONS = [  # (name, original text, mutated text, which occurrence to edit)
    ("shift sign", "y[i] = (s - c * x[i]) / d;", "y[i] = (s + c * x[i]) / d;", 0),
    ("scale dropped", "y[i] = (s - c * x[i]) / d;", "y[i] = (s - c * x[i]);", 0),
    ("gather from the row instead of the column", "s += val[k] * x[ci[k]];", "s += val[k] * x[i];", 0),
    ("recurrence sign", "vnext[i] = 2.0 * vnext[i] - vprev[i];", "vnext[i] = 2.0 * vnext[i] + vprev[i];", 0),
    ("recurrence factor dropped", "vnext[i] = 2.0 * vnext[i] - vprev[i];", "vnext[i] = vnext[i] - vprev[i];", 0),
    ("first step doubled", "z[1] = dot_neumaier(v0, vcur, n);",
     "for (int64_t i = 0; i < n; ++i) vcur[i] *= 2.0;\n                z[1] = dot_neumaier(v0, vcur, n);", 0),
    ("moment against the wrong vector", "z[k + 1] = dot_neumaier(v0, vnext, n);",
     "z[k + 1] = dot_neumaier(vcur, vnext, n);", 0),
    ("moment index off by one", "z[k + 1] = dot_neumaier(v0, vnext, n);", "z[k] = dot_neumaier(v0, vnext, n);", 0),
    ("zeta_0 not v0 . v0", "z[0] = dot_neumaier(v0, v0, n);", "z[0] = (double)n + 1.0;", 0),
    ("doubling sign", "z[2 * k] = 2.0 * dot_neumaier(vcur, vcur, n) - z[0];",
     "z[2 * k] = 2.0 * dot_neumaier(vcur, vcur, n) + z[0];", 0),
    ("probe sign from the wrong bit", "return (z >> 63) ? -1.0 : 1.0;", "return ((z >> 62) & 1) ? -1.0 : 1.0;", 0),
    ("probe counter offset dropped", "splitmix64_nth(seed, counter + 1);", "splitmix64_nth(seed, counter);", 0),
    ("SplitMix64 increment", "splitmix64_mix(seed + k * 0x9e3779b97f4a7c15ULL)",
     "splitmix64_mix(seed + k * 0x9e3779b97f4a7c13ULL)", 0),
    ("SplitMix64 shift", "z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;", "z = (z ^ (z >> 31)) * 0xbf58476d1ce4e5b9ULL;", 0),
]


def _edit(src, old, new, occurrence):
    positions, at = [], src.find(old)
    while at >= 0:
        positions.append(at)
        at = src.find(old, at + 1)
    assert positions, f"mutation target not found: {old!r}"
    at = positions[occurrence]
    return src[:at] + new + src[at + len(old):]


def _load_mutated_c(src, tmp):
    path = os.path.join(tmp, "kpm_oracle_mut.c")
    with open(path, "w") as f:
        f.write(src)
    lib_path = os.path.join(tmp, "liboracle_mut.so")
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", path, "-o", lib_path, "-lm"])
    lib = ctypes.CDLL(lib_path)
    i64, u64, i32, dbl, ptr = ctypes.c_int64, ctypes.c_uint64, ctypes.c_int, ctypes.c_double, ctypes.c_void_p
    lib.oracle_rademacher.argtypes = [u64, i64, i64, ptr]
    lib.oracle_rademacher.restype = None
    lib.oracle_rademacher_block.argtypes = [u64, i64, i32, i64, ptr]
    lib.oracle_rademacher_block.restype = None
    lib.oracle_splitmix64_nth.argtypes = [u64, u64]
    lib.oracle_splitmix64_nth.restype = u64
    for fn in (lib.oracle_moments, lib.oracle_moments_doubling):
        fn.argtypes = [i64, ptr, ptr, ptr, dbl, dbl, i32, i32, u64, i64, ptr, i32]
        fn.restype = i32
    return lib


# ---------------------------------------------------------------- Python functions
SLQ_PINS = ("test_oracle_slq.py", "test_oracle_haydock.py")
PY_MUTATIONS = [  # (name, module, function, original text, mutated text, pin files)
    ("rescale half-width dropped", oracle, "rescale", "0.5 * (ub - lb)", "(ub - lb)", CORE),
    ("normalisation by n dropped", oracle, "normalize", "range(zeta.shape[1])]) / (n * nvec)",
     "range(zeta.shape[1])]) / nvec", CORE),
    ("Jackson angle", oracle, "jackson", "a = math.pi / (M + 2)", "a = math.pi / (M + 1)", CORE),
    ("Jackson weight", oracle, "jackson", "(1.0 - k / (M + 2))", "(1.0 - k / (M + 1))", CORE),
    ("Jackson sine term sign", oracle, "jackson", "+ (1.0 / (M + 2)) * math.cos(a)",
     "- (1.0 / (M + 2)) * math.cos(a)", CORE),
    ("density factor 2 dropped", oracle, "dos_scaled", "np.where(np.arange(M + 1) == 0, 1.0, 2.0) / math.pi",
     "np.ones(M + 1) / math.pi", CORE),
    ("density weight 1/sqrt(1 - t^2) dropped", oracle, "dos_scaled", "/ np.sqrt(1.0 - ti * ti)", "", CORE),
    ("density units 1/d dropped", oracle, "dos", "(np.asarray(x) - c) / d) / d", "(np.asarray(x) - c) / d)", CORE),
    ("bin antiderivative sign", oracle, "dos_bins", "g[0] * mu[0] * (-th)", "g[0] * mu[0] * th", CORE),
    ("blurred density factor 2 dropped", oracle, "blurred_kpm",
     "np.where(np.arange(M + 1) == 0, 1.0, 2.0) * g * mu", "g * mu", CORE),
    ("Gaussian variance", oracle, "gauss", "(2.0 * sigma * sigma))", "(sigma * sigma))", CORE),
    ("Chebyshev polynomial argument", oracle, "cheb_T", "np.arccos(", "np.arcsin(", CORE),
    ("Lanczos residual from the wrong eigenvector row", oracle, "lanczos_bounds", "np.abs(Z[-1, :])",
     "np.abs(Z[0, :])", CORE),
    ("Lanczos residual sign", oracle, "lanczos_bounds", "lb0 = float(theta[0] - r[0])",
     "lb0 = float(theta[0] + r[0])", CORE),
    ("Lanczos margin inverted", oracle, "lanczos_bounds", "/ (1.0 - margin)", "* (1.0 - margin)", CORE),
    ("Lanczos breakdown merge dropped", oracle, "lanczos_bounds", "lb0, ub0 = min(lb0, g_lo), max(ub0, g_hi)",
     "pass", CORE),
    # stochastic Lanczos and Haydock (section 3.2)
    ("three-term recurrence sign", slq, "lanczos_tridiag", "- bp * Qp", "+ bp * Qp", SLQ_PINS),
    ("alpha component not removed", slq, "lanczos_tridiag", "R = W - a * Q", "R = W", SLQ_PINS),
    ("node weights from the last component", slq, "lanczos_nodes", "Z[0, :] ** 2", "Z[-1, :] ** 2", SLQ_PINS),
    ("node weights not squared", slq, "lanczos_nodes", "Z[0, :] ** 2", "np.abs(Z[0, :])", SLQ_PINS),
    ("breakdown rule dropped", slq, "steps_used", "if beta[l, k] <= BREAKDOWN_REL * scale:", "if False:",
     SLQ_PINS),
    ("mean over probes dropped", slq, "lanczos_dos", "return out / theta.shape[0]", "return out", SLQ_PINS),
    ("Haydock sign", slq, "haydock_dos", "out += -g.imag / math.pi", "out += g.imag / math.pi", SLQ_PINS),
    ("Haydock lower diagonal dropped", slq, "haydock_dos", "np.diag(off, 1) + np.diag(off, -1)",
     "np.diag(off, 1)", SLQ_PINS),
    ("Haydock scale d dropped", slq, "haydock_dos", "np.diag(c + d * alpha[l, :k])", "np.diag(c + alpha[l, :k])",
     SLQ_PINS),
    # Legendre expansions and DGL (section 3.1.3, Appendix B)
    ("Legendre recurrence coefficient", dgl, "legendre_moments_per_vector", "- k / (k + 1) * Vp",
     "- k / (k + 2) * Vp", ("test_oracle_dgl.py",)),
    ("gamma_0 constant", dgl, "dgl_gamma", "math.sqrt(math.pi / 2.0)", "math.sqrt(math.pi)",
     ("test_oracle_dgl.py",)),
    ("gamma recurrence t term", dgl, "dgl_gamma", "+ t * g[k])", "- t * g[k])", ("test_oracle_dgl.py",)),
    ("DGL weight k + 1/2", dgl, "dgl_dos", "(k + 0.5) * g * mu[:m + 1]", "k * g * mu[:m + 1]",
     ("test_oracle_dgl.py",)),
    ("Legendre density weight k + 1/2", dgl, "legendre_dos", "(np.arange(M + 1) + 0.5)", "np.arange(M + 1)",
     ("test_oracle_dgl.py",)),
    # density functionals (sections 2, 4.3)
    ("heat capacity square dropped", functional, "heat_capacity_g", "(h / np.sinh(h)) ** 2", "(h / np.sinh(h))",
     ("test_oracle_functional.py",)),
    ("KPM functional factor 2 dropped", functional, "functional_kpm",
     "w = w * np.where(np.arange(M + 1) == 0, 1.0, 2.0)", "w = w", ("test_oracle_functional.py",)),
    ("Lanczos functional mean dropped", functional, "functional_lanczos", "/ theta.shape[0])", ")",
     ("test_oracle_functional.py",)),
    # damping network
    ("GELU derivative sign", mlp, "gelu_grad", "+ u * np.exp(", "- u * np.exp(", ("test_oracle_mlp.py",)),
    ("sigmoid derivative dropped", mlp, "mlp_backward", "dz3 = dg * g * (1.0 - g)", "dz3 = dg * g",
     ("test_oracle_mlp.py",)),
    ("first layer through the second layer's input", mlp, "mlp_backward", 'dz1 = dh1 * gelu_grad(cache["z1"])',
     'dz1 = dh1 * gelu_grad(cache["z2"])', ("test_oracle_mlp.py",)),
    ("g_0 not fixed to 1", mlp, "mlp_forward", "g[:, 0] = 1.0", "pass", ("test_oracle_mlp.py",)),
    ("blur operator factor 2 dropped", mlp, "blur_operator", "w = np.where(np.arange(nmom) == 0, 1.0, 2.0)",
     "w = np.ones(nmom)", ("test_oracle_mlp.py",)),
    ("Adam second-moment bias correction", mlp, "adam_step", "v_hat = v_t / (1.0 - beta2 ** t)",
     "v_hat = v_t / (1.0 - beta1 ** t)", ("test_oracle_mlp.py",)),
    ("Adam first-moment decay", mlp, "adam_step", "(1.0 - beta1) * g", "(1.0 - beta2) * g",
     ("test_oracle_mlp.py",)),
]


def _apply_py(monkeypatch, module, name, old, new):
    orig = getattr(module, name)
    src = textwrap.dedent(inspect.getsource(orig))
    assert src.count(old) == 1, f"mutation target must occur once in {name}: {old!r}"
    ns = dict(vars(module))
    exec(compile(src.replace(old, new), f"<mutated {name}>", "exec"), ns)
    for mod in MODULES:  # the function and every alias of it in the package
        for attr, val in list(vars(mod).items()):
            if val is orig:
                monkeypatch.setattr(mod, attr, ns[name])


def test_unmutated_oracle_passes_every_pin():
    files = sorted({f for m in PY_MUTATIONS for f in m[5]} | set(CORE))
    assert _failing_pins(files) == []


@pytest.mark.parametrize("name,old,new,occurrence", C_MUTATIONS, ids=[m[0] for m in C_MUTATIONS])
def test_c_mutation_is_caught(monkeypatch, name, old, new, occurrence):
    with open(C_SRC) as f:
        src = f.read()
    with tempfile.TemporaryDirectory() as tmp:
        monkeypatch.setattr(oracle, "_lib", _load_mutated_c(_edit(src, old, new, occurrence), tmp))
        failed = _failing_pins(CORE)
    assert failed, f"no pin fails under the mutation '{name}'"


@pytest.mark.parametrize("name,module,func,old,new,pin_files", PY_MUTATIONS, ids=[m[0] for m in PY_MUTATIONS])
def test_python_mutation_is_caught(monkeypatch, name, module, func, old, new, pin_files):
    _apply_py(monkeypatch, module, func, old, new)
    failed = _failing_pins(pin_files)
    assert failed, f"no pin fails under the mutation '{name}'"
