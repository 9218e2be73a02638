"""The C-ABI library: it loads, exports every entry point that include/crl.h
declares, and rejects bad arguments on the host before touching a device.
No GPU needed."""
import ctypes as C
import os
import re

import pytest

from paper_2408_11052_amd import _lib
from synthetic import workloads as WL

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "crl.h")


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"CRL_API\s+[\w\s\*]+?\b(crl_\w+)\s*\(", src)))


def test_header_declares_the_hot_path_calls():
    names = _declared()
    for n in ("crl_sample_relabel", "crl_critic_fwd", "crl_critic_bwd", "crl_adam_step",
              "crl_critic_bwd_adam", "crl_actor_step", "crl_actor_step_adam"):
        assert n in names


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing
    # and the Python binding declares exactly these
    assert sorted(_lib.SIGNATURES) == _declared()


def test_only_crl_symbols_are_exported():
    out = os.popen(f"nm -D --defined-only {_lib.LIB_PATH}").read().split("\n")
    syms = [l.split()[-1] for l in out if l.strip() and l.split()[1] in ("T", "W")]
    assert syms and all(s.startswith("crl_") or s.startswith("_") for s in syms), syms


def _create(**kw):
    from paper_2408_11052_amd.critic import make_config
    cfg = make_config(WL.SMALL_RELU)
    for k, v in kw.items():
        setattr(cfg, k, v)
    ctx = C.c_void_p()
    rc = _lib.lib().crl_create(C.byref(cfg), C.byref(ctx))
    return rc, _lib.lib().crl_last_error().decode()


@pytest.mark.parametrize("field,value,msg", [
    ("batch", 0, "batch"),
    ("hidden", 100, "hidden"),
    ("hidden", 2048, "hidden"),
    ("repr_dim", 12, "repr_dim"),
    ("goal_lo", 28, "goal slice"),
    ("energy", 7, "energy"),
    ("loss", 9, "loss"),
    ("energy", -1, "energy"),
    ("discount", 1.0, "discount"),
    ("discount", 0.0, "discount"),
    ("max_episode_len", 1, "max_episode_len"),
    ("ln_eps", 0.0, "ln_eps"),
    ("logsumexp_penalty", -1.0, "logsumexp_penalty"),
    ("n_hidden", 0, "n_hidden"),
])
def test_create_rejects_bad_config_on_host(field, value, msg):
    rc, err = _create(**{field: value})
    assert rc == _lib.CRL_EINVAL
    assert msg in err


@pytest.mark.parametrize("fields,msg", [
    ({"actor_n_hidden": 2, "actor_hidden": 100}, "actor_hidden"),
    ({"actor_n_hidden": 2, "actor_hidden": 2048}, "actor_hidden"),
    ({"actor_n_hidden": 17, "actor_hidden": 64}, "actor_n_hidden"),
    ({"actor_n_hidden": 0, "actor_hidden": 64}, "actor_hidden"),
    ({"actor_n_hidden": 2, "actor_hidden": 64, "act_dim": 0}, "act_dim"),
    ({"actor_n_hidden": 2, "actor_hidden": 64, "target_entropy": float("nan")},
     "target_entropy"),
])
def test_create_rejects_bad_policy_config(fields, msg):
    rc, err = _create(**fields)
    assert rc == _lib.CRL_EINVAL
    assert msg in err


def test_policy_config_fields_follow_the_workload():
    from paper_2408_11052_amd.critic import make_config
    cfg = make_config(WL.FULL_UPDATE_B4096)
    assert (cfg.actor_n_hidden, cfg.actor_hidden) == (4, 1024)
    assert cfg.target_entropy == -WL.FULL_UPDATE_B4096.act_dim
    cfg = make_config(WL.DOT_B4096_BF16)
    assert (cfg.actor_n_hidden, cfg.actor_hidden, cfg.target_entropy) == (0, 0, 0.0)


def test_ctypes_structs_match_the_c_header(tmp_path):
    """Size and field offsets of crl_config / crl_layer_info as the C compiler
    lays them out from include/crl.h, against the ctypes mirror."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    fields = [f for f, _ in _lib.crl_config._fields_]
    lines = [f'printf("crl_config %zu\\n", sizeof(crl_config));']
    lines += [f'printf("crl_config.{f} %zu\\n", offsetof(crl_config, {f}));' for f in fields]
    lines += ['printf("crl_layer_info %zu\\n", sizeof(crl_layer_info));']
    src = tmp_path / "layout.c"
    src.write_text("#include <stddef.h>\n#include <stdio.h>\n#include \"crl.h\"\n"
                   "int main(void) {\n" + "\n".join(lines) + "\nreturn 0; }\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = dict(l.rsplit(" ", 1) for l in subprocess.run(
        [str(exe)], check=True, capture_output=True, text=True).stdout.splitlines())
    assert int(out["crl_config"]) == C.sizeof(_lib.crl_config)
    for f in fields:
        assert int(out[f"crl_config.{f}"]) == getattr(_lib.crl_config, f).offset, f
    assert int(out["crl_layer_info"]) == C.sizeof(_lib.crl_layer_info)


def test_create_rejects_unsupported_combinations():
    rc, err = _create(logits=1)  # fused logits with FP32 tiles
    assert rc == _lib.CRL_EUNSUPPORTED and "BF16" in err
    rc, err = _create(logits=1, precision=1, repr_dim=48)
    assert rc == _lib.CRL_EUNSUPPORTED and "repr_dim" in err
    # the L1 energy is not a product, the pairwise objectives need the matrix
    rc, err = _create(logits=1, precision=1, energy=_lib.ENERGY["l1"])
    assert rc == _lib.CRL_EUNSUPPORTED and "L1" in err
    for loss in ("fb", "dpo", "ipo", "sppo"):
        rc, err = _create(logits=1, precision=1, loss=_lib.LOSS[loss])
        assert rc == _lib.CRL_EUNSUPPORTED and "pairwise" in err
    rc, err = _create(energy=_lib.ENERGY["l1"], repr_dim=512)
    assert rc == _lib.CRL_EUNSUPPORTED and "L1" in err


def test_enums_follow_the_header():
    src = open(HEADER).read()
    for name, v in _lib.ENERGY.items():
        key = {"l2sq": "L2SQ"}.get(name, name.upper())
        assert re.search(rf"CRL_ENERGY_{key}\s*=\s*{v}\b", src), name
    for name, v in _lib.LOSS.items():
        key = {"fwd_infonce": "FWD", "symmetric_infonce": "SYM", "bwd_infonce": "BWD"}.get(
            name, name.upper())
        assert re.search(rf"CRL_LOSS_{key}\s*=\s*{v}\b", src), name
    assert re.search(r"CRL_ENONFINITE\s*=\s*-4", src)


def test_reserved_fields_must_be_zero():
    from paper_2408_11052_amd.critic import make_config
    cfg = make_config(WL.SMALL_RELU)
    cfg.reserved[1] = 1
    ctx = C.c_void_p()
    assert _lib.lib().crl_create(C.byref(cfg), C.byref(ctx)) == _lib.CRL_EINVAL


def test_null_arguments_rejected_without_device():
    L = _lib.lib()
    assert L.crl_create(None, None) == _lib.CRL_EINVAL
    assert L.crl_adam_step(None, None, None, None, None, 10, None, 1e-3, 0.9, 0.999, 1e-8,
                           None) == _lib.CRL_EINVAL
    assert L.crl_counter_add(None, 1, None) == _lib.CRL_EINVAL
    assert L.crl_cast_bf16(None, None, 4, None) == _lib.CRL_EINVAL
    assert L.crl_sample_relabel(None, None, None, 1, 2, 0, None, None, None, None, None,
                                None) == _lib.CRL_EINVAL
    assert L.crl_actor_step(None, None, None, None, None, None, None, None, None, 0, None,
                            None, None, None, None, None) == _lib.CRL_EINVAL
    n64 = C.c_int64()
    assert L.crl_actor_param_count(None, C.byref(n64)) == _lib.CRL_EINVAL
    assert L.crl_infonce_fwd(None, None, None, None, None, None) == _lib.CRL_EINVAL
    assert L.crl_infonce_bwd(None, None, None, None, None, None, None) == _lib.CRL_EINVAL
    assert L.crl_check_finite(None, None) == _lib.CRL_EINVAL
    assert L.crl_critic_bwd_adam(None, None, None, None, None, None, None, None, None, None,
                                 1e-3, 0.9, 0.999, 1e-8, None) == _lib.CRL_EINVAL
    assert L.crl_actor_step_adam(None, None, None, None, None, None, None, None, None, 0, None,
                                 None, None, None, None, None, None, None, 1e-3, 0.9, 0.999,
                                 1e-8, None) == _lib.CRL_EINVAL
    n = C.c_int32()
    assert L.crl_timing_count(C.byref(n)) == _lib.CRL_OK


def test_adam_rejects_misaligned_and_bad_hyperparameters():
    L = _lib.lib()
    buf = (C.c_float * 64)()
    base = C.addressof(buf)
    base16 = (base + 15) // 16 * 16
    p = C.c_void_p(base16)
    mis = C.c_void_p(base16 + 4)
    step = C.c_void_p(base16)
    assert L.crl_adam_step(mis, p, p, p, None, 4, step, 1e-3, 0.9, 0.999, 1e-8,
                           None) == _lib.CRL_EINVAL
    assert L.crl_adam_step(p, p, p, p, None, 4, step, 1e-3, 1.5, 0.999, 1e-8,
                           None) == _lib.CRL_EINVAL
    assert L.crl_adam_step(p, p, p, p, None, -1, step, 1e-3, 0.9, 0.999, 1e-8,
                           None) == _lib.CRL_EINVAL
    assert "Adam" in L.crl_last_error().decode() or "n must" in L.crl_last_error().decode()
