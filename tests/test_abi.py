"""The C-ABI library loads and exports every entry point of include/mpixs.h
(CPU only: no call here touches the GPU)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mpixs.h")
LIB = os.path.join(ROOT, "paper_2208_13707_amd", "libmpixs.so")
HEADERS = {  # header -> library that must export its functions
    "mpixs.h": LIB,
    "mpixs_debug.h": LIB,
    "mpixs_driver.h": os.path.join(ROOT, "paper_2208_13707_amd", "libmpixs_driver.so"),
}


def declared(header="mpixs.h"):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mpixs_[a-z_0-9]+)\s*\(", text)))


def test_every_header_is_covered():
    assert sorted(HEADERS) == sorted(f for f in os.listdir(os.path.join(ROOT, "include"))
                                     if f.endswith(".h"))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libmpixs.so is not built (run __graft_entry__.build())")
    from paper_2208_13707_amd import mpixs as M
    return M.lib()


def test_header_declares_the_boundary():
    names = declared()
    for required in ("mpixs_stream_create", "mpixs_stream_free", "mpixs_comm_create_with_stream",
                     "mpixs_send_enqueue", "mpixs_recv_enqueue", "mpixs_isend_enqueue",
                     "mpixs_wait_enqueue", "mpixs_allreduce_enqueue", "mpixs_info_set_hex"):
        assert required in names


@pytest.mark.parametrize("header", sorted(HEADERS))
def test_every_declared_symbol_is_exported(lib, header):
    path = HEADERS[header]
    assert os.path.exists(path), f"{path} is not built"
    out = subprocess.run(["nm", "-D", "--defined-only", path], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (mpixs_[a-z_0-9]+)", out))
    missing = [n for n in declared(header) if n not in exported]
    assert not missing, missing


def test_binding_covers_the_header():
    from paper_2208_13707_amd import mpixs as M
    missing = [n for n in declared() if n not in M.SIGNATURES or not hasattr(M, n)]
    assert not missing, missing


def test_error_strings(lib):
    from paper_2208_13707_amd import mpixs as M
    for code, name in M.ERR_NAMES.items():
        assert M.mpixs_error_string(code) == name


def test_info_hex_encoding(lib):
    """Info objects are host-only: the hex text of a binary value (§3.2)."""
    from paper_2208_13707_amd import mpixs as M
    rc, info = M.mpixs_info_create()
    assert rc == 0
    assert M.mpixs_info_set(info, "type", "hipStream_t") == 0
    assert M.mpixs_info_set_hex(info, "value", bytes([0x00, 0x1f, 0xa0, 0xff])) == 0
    assert M.mpixs_info_get(info, "value") == (0, "001fa0ff")
    assert M.mpixs_info_get(info, "type") == (0, "hipStream_t")
    assert M.mpixs_info_get(info, "nope") == (0, None)
    assert M.mpixs_info_free(info) == 0


def test_bad_batch_schedule_is_rejected_before_any_gpu_call(lib):
    """Invalid batch schedules fail with ERR_ARG while the world is validated,
    before the library touches the device (so this runs without a GPU)."""
    from paper_2208_13707_amd import mpixs as M
    for fields in ({"batch_tile": 300}, {"batch_tile": 8192}, {"batch_graph": 2},
                   {"batch_max_wg": 1 << 21}, {"batch_sync": 2}, {"batch_sync": -1},
                   {"batch_sync": 1, "batch_graph": 1}):
        c = M.Config()
        for field, value in fields.items():
            setattr(c, field, value)
        rc, w = M.mpixs_world_create(2, c)
        assert M.errname(rc) == "ERR_ARG" and not w, fields


def test_structs_match_the_header(tmp_path):
    """Every struct the bindings marshal has the header's size and field
    offsets (compiled from include/ with the host C compiler)."""
    import ctypes
    import shutil
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    from paper_2208_13707_amd import driver as D
    from paper_2208_13707_amd import mpixs as M
    ct = [("mpixs_config", M.Config), ("mpixs_status", M.Status), ("mpixs_stats", M.Stats),
          ("mpixs_trace_event", M.TraceEvent),
          ("mpixs_drv_thread", D.DrvThread), ("mpixs_drv_result", D.DrvResult)]
    npy = [("mpixs_drv_op", D.OP_DTYPE), ("mpixs_drv_req", D.REQ_DTYPE),
           ("mpixs_drv_req_result", D.RES_DTYPE)]
    want = {}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "mpixs.h"',
             '#include "mpixs_driver.h"', "int main(void) {"]
    for cname, cls in ct:
        want[cname] = ctypes.sizeof(cls)
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            want[f"{cname}.{f}"] = getattr(cls, f).offset
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    for cname, dt in npy:
        want[cname] = dt.itemsize
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f in dt.names:
            want[f"{cname}.{f}"] = dt.fields[f][1]
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run(["gcc", "-I", inc, str(src), "-o", str(exe)], check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                        text=True).stdout.splitlines())
    assert {k: int(v) for k, v in got.items()} == want


def test_one_hip_runtime_whatever_is_loaded_first():
    """Loading the library first still leaves one HIP runtime in the process
    (torch's, which the binding loads before the library)."""
    code = ("from paper_2208_13707_amd import mpixs as M\n"
            "from paper_2208_13707_amd import driver as D\n"
            "M.lib(); D._hiplib()\n"
            "import torch\n"
            "maps = open('/proc/self/maps').read().split(chr(10))\n"
            "libs = {l.split()[-1] for l in maps if 'libamdhip64' in l}\n"
            "print(len(libs))\n")
    out = subprocess.run(["python", "-c", code], cwd=ROOT, capture_output=True, text=True,
                         timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    assert out.stdout.strip().splitlines()[-1] == "1"
