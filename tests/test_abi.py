"""The C ABI library loads without a GPU and exports every entry point the header declares."""
import os
import re

import paper_2404_17084_amd as em

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "exactmap.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char \*|void|int64_t)\s*\*?\s*(map_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_entry_points():
    names = declared_functions()
    for must in ("map_init", "map_shutdown", "map_last_error", "map_pairs", "map_particles"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = em.load()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_has_same_names():
    missing = [n for n in declared_functions() if not callable(getattr(em, n, None))]
    assert not missing, missing


def test_product_path_never_touches_the_oracle():
    pkg = os.path.join(ROOT, "paper_2404_17084_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text and "exact_oracle" not in text, f


def test_init_without_gpu_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        return
    try:
        em.map_init(0)
    except em.MapError as e:
        assert e.code in (em.MAP_EDEVICE, em.MAP_EINVAL)
    else:
        raise AssertionError("map_init succeeded without a device")
