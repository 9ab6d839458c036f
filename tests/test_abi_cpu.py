"""CPU checks of the C-ABI library: it loads, exports every function that
include/lbm.h declares, and the ctypes structures agree with the header's
field lists. No compute call is made (no GPU here)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", text)))


def declared_struct_fields(name):
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct \{([^{}]*)\}\s*" + name + ";", text, re.S).group(1)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        names = decl.split(None, 1)[1] if not decl.startswith("const") else decl.split(None, 2)[2]
        for n in names.split(","):
            fields.append(re.sub(r"[\*\s]|\[.*\]", "", n))
    return fields


def test_library_exports_every_declared_function():
    from paper_1407_4524_amd import lbm
    L = lbm.lib()
    names = declared_functions()
    assert "lbm_step" in names and "lbm_force_torque" in names and len(names) >= 12
    for n in names:
        assert hasattr(L, n), f"{n} declared in include/lbm.h but not exported"
    assert set(names) == set(lbm.EXPORTS)


@pytest.mark.parametrize("cname,pyname", [("lbm_domain_desc", "DomainDesc"), ("lbm_body_desc", "BodyDesc"),
                                          ("lbm_batch_config", "BatchConfig"),
                                          ("lbm_sweep_config", "SweepConfig")])
def test_ctypes_structs_follow_header(cname, pyname):
    from paper_1407_4524_amd import lbm
    py = [f[0] for f in getattr(lbm, pyname)._fields_]
    c = declared_struct_fields(cname)
    assert c == py


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_1407_4524_amd import lbm
    monkeypatch.setattr(lbm, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(lbm, "_lib", None)
    with pytest.raises(ImportError):
        lbm.lib()


def test_bench_refuses_more_than_one_gpu():
    """the benchmark runs on one GPU only and says so, before touching any device"""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=root)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout.strip() == ""


@pytest.mark.parametrize("kw,msg", [
    (dict(nx=2), "each axis needs >= 3 nodes"),
    (dict(lattice="D3Q19", nz=2), "each axis needs >= 3 nodes"),
    (dict(ny=32001), "axis longer than 32000 nodes"),
    (dict(tau=0.5), "tau must exceed 1/2"),
    (dict(rho0=0.0), "rho0 must be positive"),
    (dict(faces=("periodic", "wall", "wall", "wall", "periodic", "periodic")), "periodic faces come in pairs"),
    (dict(faces=("outlet", "outlet", "wall", "wall", "periodic", "periodic")), "inlet only on -x"),
    (dict(faces=("wall", "wall", "inlet", "wall", "periodic", "periodic")), "inlet/outlet faces only along x"),
    (dict(split_schedule=2), "split_schedule is -1, 0 or 1"),
    (dict(split_schedule=-2), "split_schedule is -1, 0 or 1"),
])
def test_invalid_domain_rejected_on_the_host(kw, msg):
    """The descriptor checks run before any HIP call: each invalid setting
    gives LBM_E_INVAL and its message from lbm_create_domain and from
    lbm_footprint_bytes, without a GPU."""
    import ctypes as C
    from paper_1407_4524_amd import Domain, lbm
    with pytest.raises(lbm.LbmError) as e:
        Domain(**kw)
    assert e.value.status == -1 and msg in str(e.value)
    d = lbm.domain_desc(**kw)
    n = C.c_size_t(0)
    assert lbm.lib().lbm_footprint_bytes(C.byref(d), C.byref(n)) == -1
    assert msg in lbm.lib().lbm_last_error().decode()


def test_footprint_follows_the_layout():
    """lbm_footprint_bytes (host arithmetic only) grows with the storage
    width and the lattice, and covers both population buffers."""
    import ctypes as C
    from paper_1407_4524_amd import lbm

    def fp(**kw):
        n = C.c_size_t(0)
        assert lbm.lib().lbm_footprint_bytes(C.byref(lbm.domain_desc(**kw)), C.byref(n)) == 0
        return n.value

    nx, ny = 500, 300
    f64, f32, f16 = (fp(nx=nx, ny=ny, storage=s) for s in ("f64", "f32", "f16"))
    assert f64 > f32 > f16
    assert f32 >= 2 * 9 * nx * ny * 4 and f16 >= 2 * 9 * nx * ny * 2
    assert fp(lattice="D3Q19", nx=40, ny=30, nz=20) >= 2 * 19 * 40 * 30 * 20 * 4


def test_hbm_traffic_scaling(tmp_path):
    """The counter arithmetic behind the bench line's traffic figure: each
    counter is scaled by its reading for a plain copy of known size, and the
    kernel's most frequent launch shape is the one summarised."""
    from paper_1407_4524_amd import hbm_traffic as H

    def write(path, counter, rows):
        with open(path, "w") as fh:
            fh.write("Kernel_Name,Grid_Size,Counter_Name,Counter_Value\n")
            for name, grid, v in rows:
                fh.write(f"{name},{grid},{counter},{v}\n")

    k = "void lbm::k_stream_collide<D2Q9>(float const*)"
    copy = H.COPY_KERNEL
    fetch, wr = tmp_path / "f.csv", tmp_path / "w.csv"
    # copy of 1 MiB in total: the fetch counter sees half of its 512 KiB read, the write counter all
    write(fetch, "FETCH_SIZE", [(k, 4096, 100.0), (k, 4096, 102.0), (k, 64, 9.0), (copy, 256, 256.0)])
    write(wr, "WRITE_SIZE", [(k, 4096, 200.0), (k, 4096, 200.0), (k, 64, 9.0), (copy, 256, 512.0)])
    r = H.summarize(str(fetch), str(wr), "void lbm::k_stream_collide", 1 << 20)
    assert r["grid"] == 4096 and r["dispatches"] == [2, 2]
    assert r["fetch_scale"] == 0.5 and r["write_scale"] == 1.0
    assert r["hbm_read_bytes_per_launch"] == round(101.0 * 1024 / 0.5)
    assert r["hbm_write_bytes_per_launch"] == 200 * 1024
    assert r["hbm_bytes_per_launch"] == r["hbm_read_bytes_per_launch"] + r["hbm_write_bytes_per_launch"]
    assert r["kernel_source_sha256_16"] == H.kernel_source_hash()
