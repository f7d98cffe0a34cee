"""Host-side checks of the C ABI (no GPU needed): the HIP library loads,
exports every function include/mkf.h declares, and the Python binding's
structures have the layout a C compiler gives the header's."""
import ast
import ctypes as C
import os
import sys
import subprocess
import tempfile

import pytest

from paper_1702_06359_amd import abi, build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def libpath():
    if not os.path.exists(abi.LIB_PATH):
        build.build(force=True)
    return abi.LIB_PATH


def test_library_exports_every_declared_function(libpath):
    names = abi.header_functions()
    assert len(names) >= 20
    L = C.CDLL(libpath)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    # and the binding prototypes every one of them
    assert sorted(abi._PROTOS) == names


def test_exported_symbols_are_unmangled_c(libpath):
    out = subprocess.run(["nm", "-D", "--defined-only", libpath], capture_output=True, text=True).stdout
    syms = {line.split()[-1] for line in out.splitlines() if line.strip()}
    for n in abi.header_functions():
        assert n in syms


def test_binding_struct_layouts_match_the_header():
    structs = {
        "mkf_config": (abi.Config, ["n_layers", "flags", "layer_r", "layer_half_z", "layer_x0", "bz", "chi2_cut",
                                    "mass", "layer_kind", "layer_z", "layer_rmin", "sigma_r", "layer_thickness"]),
        "mkf_allocator": (abi.Allocator, ["alloc", "free", "user"]),
        "mkf_event": (abi.Event, ["n_layers", "n_seeds", "n_tracks", "n_hits", "hit_xyz", "seed_par", "seed_cov",
                                  "seed_hits", "track_par", "track_cov", "track_hits"]),
        "mkf_tracks": (abi.Tracks, ["n", "par", "cov", "hits", "n_hits", "n_holes", "chi2", "ndof", "status"]),
        "mkf_tuning": (abi.Tuning, ["lanes_per_seed", "waves_per_block", "bins_phi", "bins_z", "persistent",
                                    "blocks_per_cu"]),
        "mkf_build_stats": (abi.BuildStats, ["cand_layers", "chi2_evals", "accepted", "updates", "hits_scanned"]),
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{ROOT}/include/mkf.h"', "int main(void){"]
    for cname, (_, fields) in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f in fields:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append(f'printf("MKF_MAX_LAYERS %d\\nMKF_MAX_CANDS %d\\n", MKF_MAX_LAYERS, MKF_MAX_CANDS);')
    lines.append("return 0;}")
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "layout.c")
        exe = os.path.join(d, "layout")
        with open(src, "w") as f:
            f.write("\n".join(lines))
        subprocess.check_call(["gcc", "-std=c11", "-Wall", "-Werror", "-o", exe, src])
        out = subprocess.check_output([exe], text=True)
    got = {}
    for line in out.splitlines():
        parts = line.split()
        got[tuple(parts[:-1])] = int(parts[-1])
    assert got[("MKF_MAX_LAYERS",)] == abi.MAX_LAYERS
    assert got[("MKF_MAX_CANDS",)] == abi.MAX_CANDS
    for cname, (cls, fields) in structs.items():
        assert got[(cname, "size")] == C.sizeof(cls), cname
        for f in fields:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)


def test_header_compiles_as_c_and_cpp():
    with tempfile.TemporaryDirectory() as d:
        for lang, comp in (("c", "gcc"), ("cpp", "g++")):
            src = os.path.join(d, f"h.{lang}")
            with open(src, "w") as f:
                f.write(f'#include "{ROOT}/include/mkf.h"\nint main(void){{return (int)MKF_OK;}}\n')
            subprocess.check_call([comp, "-Wall", "-Werror", "-o", os.path.join(d, f"h_{lang}"), src])


def test_create_without_gpu_fails_cleanly(libpath):
    """With no GPU visible mkf_create reports MKF_E_DEVICE instead of crashing."""
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is visible")
    except ImportError:
        pass
    from paper_1702_06359_amd import synth
    cfg = abi.config_from_geometry(synth.Geometry())
    h = C.c_void_p()
    st = abi.lib().mkf_create(C.byref(cfg), None, None, C.byref(h))
    assert st == abi.E_DEVICE
    assert abi.last_error()


def test_invalid_config_rejected_before_device_work(libpath):
    from paper_1702_06359_amd import synth
    cfg = abi.config_from_geometry(synth.Geometry(), max_cands=9)
    h = C.c_void_p()
    assert abi.lib().mkf_create(C.byref(cfg), None, None, C.byref(h)) == abi.E_INVALID
    cfg = abi.config_from_geometry(synth.Geometry())
    cfg.layer_r[3] = cfg.layer_r[2]
    assert abi.lib().mkf_create(C.byref(cfg), None, None, C.byref(h)) == abi.E_INVALID
    assert "radii" in abi.last_error()


def test_library_shares_one_hip_runtime_with_torch(libpath):
    """Loading the library before anything imports torch must still leave a
    single HIP runtime in the process (torch's), since torch's streams and
    device memory are passed to the library."""
    pytest.importorskip("torch")
    code = ("from paper_1702_06359_amd import abi; abi.lib(); import torch; "
            "print(sorted({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}))")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300,
                         cwd=os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    assert out.returncode == 0, out.stderr
    libs = ast.literal_eval(out.stdout.strip().splitlines()[-1])
    assert len(libs) == 1, libs
