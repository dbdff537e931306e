"""Guard on the compiled kernels' private (scratch) memory: every kernel of
libpdd's gfx950 code object uses exactly the listed private segment and
spilled VGPRs, and every kernel not listed uses none.  A change in a
kernel's spills or stack (the class of code behind a wrong result that an
earlier, spill-heavy form of the float64 network gradient gave) then fails
here, on the CPU, and the new figures must be reviewed and listed.

The figures are read from the AMDGPU metadata notes of the library's own
code objects (clang-offload-bundler and llvm-readelf of the build here)."""
import os
import re
import subprocess

import pytest
import yaml

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2301_05780_amd", "libpdd.so")
LLVM = "/opt/rocm/llvm/bin"

# mangled kernel name: (private_segment_fixed_size bytes, vgpr_spill_count)
LISTED = {
    "_ZN3pdd12_GLOBAL__N_111k_calibrateILi0ELb0ELb0EEEvNS0_7CalArgsE": (136, 0),
    "_ZN3pdd12_GLOBAL__N_111k_calibrateILi0ELb0ELb1EEEvNS0_7CalArgsE": (136, 0),
    "_ZN3pdd12_GLOBAL__N_111k_calibrateILi0ELb1ELb0EEEvNS0_7CalArgsE": (136, 0),
    "_ZN3pdd12_GLOBAL__N_111k_calibrateILi0ELb1ELb1EEEvNS0_7CalArgsE": (136, 0),
    "_ZN3pdd12_GLOBAL__N_111k_calibrateILi1ELb0ELb0EEEvNS0_7CalArgsE": (136, 0),
    "_ZN3pdd12_GLOBAL__N_111k_calibrateILi1ELb0ELb1EEEvNS0_7CalArgsE": (136, 0),
    "_ZN3pdd12_GLOBAL__N_111k_calibrateILi1ELb1ELb0EEEvNS0_7CalArgsE": (136, 0),
    "_ZN3pdd12_GLOBAL__N_111k_calibrateILi1ELb1ELb1EEEvNS0_7CalArgsE": (136, 0),
    "_ZN3pdd12_GLOBAL__N_111k_calibrateILi2ELb0ELb0EEEvNS0_7CalArgsE": (136, 0),
    "_ZN3pdd12_GLOBAL__N_111k_calibrateILi2ELb0ELb1EEEvNS0_7CalArgsE": (136, 0),
    "_ZN3pdd12_GLOBAL__N_111k_calibrateILi2ELb1ELb0EEEvNS0_7CalArgsE": (136, 0),
    "_ZN3pdd12_GLOBAL__N_111k_calibrateILi2ELb1ELb1EEEvNS0_7CalArgsE": (136, 0),
    "_ZN3pdd12_GLOBAL__N_111k_calibrateILi3ELb0ELb0EEEvNS0_7CalArgsE": (136, 0),
    "_ZN3pdd12_GLOBAL__N_111k_calibrateILi3ELb0ELb1EEEvNS0_7CalArgsE": (136, 0),
    "_ZN3pdd12_GLOBAL__N_111k_calibrateILi3ELb1ELb0EEEvNS0_7CalArgsE": (136, 0),
    "_ZN3pdd12_GLOBAL__N_111k_calibrateILi3ELb1ELb1EEEvNS0_7CalArgsE": (136, 0),
    "_ZN3pdd12_GLOBAL__N_111k_calibrateILi4ELb0ELb0EEEvNS0_7CalArgsE": (136, 0),
    "_ZN3pdd12_GLOBAL__N_111k_calibrateILi4ELb0ELb1EEEvNS0_7CalArgsE": (136, 0),
    "_ZN3pdd12_GLOBAL__N_111k_calibrateILi4ELb1ELb0EEEvNS0_7CalArgsE": (136, 0),
    "_ZN3pdd12_GLOBAL__N_111k_calibrateILi4ELb1ELb1EEEvNS0_7CalArgsE": (136, 0),
    "_ZN3pdd12_GLOBAL__N_111k_calibrateILi5ELb0ELb0EEEvNS0_7CalArgsE": (136, 0),
    "_ZN3pdd12_GLOBAL__N_111k_calibrateILi5ELb0ELb1EEEvNS0_7CalArgsE": (136, 0),
    "_ZN3pdd12_GLOBAL__N_111k_calibrateILi5ELb1ELb0EEEvNS0_7CalArgsE": (136, 0),
    "_ZN3pdd12_GLOBAL__N_111k_calibrateILi5ELb1ELb1EEEvNS0_7CalArgsE": (136, 0),
    "_ZN3pdd12_GLOBAL__N_111k_calibrateILi6ELb0ELb0EEEvNS0_7CalArgsE": (136, 0),
    "_ZN3pdd12_GLOBAL__N_111k_calibrateILi6ELb0ELb1EEEvNS0_7CalArgsE": (136, 0),
    "_ZN3pdd12_GLOBAL__N_111k_calibrateILi6ELb1ELb0EEEvNS0_7CalArgsE": (136, 0),
    "_ZN3pdd12_GLOBAL__N_111k_calibrateILi6ELb1ELb1EEEvNS0_7CalArgsE": (136, 0),
    "_ZN3pdd12_GLOBAL__N_113k_assemble_w6ILi6EEEvNS_9AsmParamsE": (92, 26),
    "_ZN3pdd12_GLOBAL__N_115k_assemble_laneILi0EEEvNS_9AsmParamsE": (20, 4),
    "_ZN3pdd12_GLOBAL__N_115k_assemble_laneILi2EEEvNS_9AsmParamsE": (32, 7),
    "_ZN3pdd12_GLOBAL__N_16k_evalILi0ELb0EEEvNS0_8EvalArgsE": (136, 0),
    "_ZN3pdd12_GLOBAL__N_16k_evalILi0ELb1EEEvNS0_8EvalArgsE": (136, 0),
    "_ZN3pdd12_GLOBAL__N_16k_evalILi1ELb0EEEvNS0_8EvalArgsE": (136, 0),
    "_ZN3pdd12_GLOBAL__N_16k_evalILi1ELb1EEEvNS0_8EvalArgsE": (136, 0),
    "_ZN3pdd12_GLOBAL__N_16k_evalILi2ELb0EEEvNS0_8EvalArgsE": (136, 0),
    "_ZN3pdd12_GLOBAL__N_16k_evalILi2ELb1EEEvNS0_8EvalArgsE": (136, 0),
    "_ZN3pdd12_GLOBAL__N_16k_evalILi3ELb0EEEvNS0_8EvalArgsE": (136, 0),
    "_ZN3pdd12_GLOBAL__N_16k_evalILi3ELb1EEEvNS0_8EvalArgsE": (136, 0),
    "_ZN3pdd12_GLOBAL__N_16k_evalILi4ELb0EEEvNS0_8EvalArgsE": (136, 0),
    "_ZN3pdd12_GLOBAL__N_16k_evalILi4ELb1EEEvNS0_8EvalArgsE": (136, 0),
    "_ZN3pdd12_GLOBAL__N_16k_evalILi5ELb0EEEvNS0_8EvalArgsE": (136, 0),
    "_ZN3pdd12_GLOBAL__N_16k_evalILi5ELb1EEEvNS0_8EvalArgsE": (136, 0),
    "_ZN3pdd12_GLOBAL__N_16k_evalILi6ELb0EEEvNS0_8EvalArgsE": (136, 0),
    "_ZN3pdd12_GLOBAL__N_16k_evalILi6ELb1EEEvNS0_8EvalArgsE": (136, 0),
}


def _kernels(tmp):
    objcopy, bundler, readelf = (os.path.join(LLVM, t) for t in ("llvm-objcopy", "clang-offload-bundler", "llvm-readelf"))
    if not all(os.path.exists(t) for t in (objcopy, bundler, readelf)) or not os.path.exists(LIB):
        pytest.skip("ROCm LLVM tools or the built library not available")
    fat = os.path.join(tmp, "fatbin.bin")
    subprocess.run([objcopy, "--dump-section", f".hip_fatbin={fat}", LIB, os.path.join(tmp, "lib.so")], check=True)
    data = open(fat, "rb").read()
    starts = [m.start() for m in re.finditer(re.escape(b"__CLANG_OFFLOAD_BUNDLE__"), data)]
    out = {}
    for n, a in enumerate(starts):
        b = starts[n + 1] if n + 1 < len(starts) else len(data)
        part, co = os.path.join(tmp, f"b{n}.bin"), os.path.join(tmp, f"co{n}.elf")
        open(part, "wb").write(data[a:b])
        subprocess.run([bundler, "--unbundle", "--type=o", "--targets=hipv4-amdgcn-amd-amdhsa--gfx950",
                        f"--input={part}", f"--output={co}"], check=True, capture_output=True)
        notes = subprocess.run([readelf, "--notes", co], check=True, capture_output=True, text=True).stdout
        y0 = notes.find("---")
        meta = yaml.safe_load(notes[y0:notes.find("...", y0)])
        for k in meta.get("amdhsa.kernels", []):
            out[k[".name"]] = (int(k.get(".private_segment_fixed_size", 0)), int(k.get(".vgpr_spill_count", 0)))
    return out


def test_private_memory_of_every_kernel_is_as_listed(tmp_path):
    got = _kernels(str(tmp_path))
    assert len(got) > 100
    changed = {k: (v, LISTED.get(k, (0, 0))) for k, v in got.items() if v != LISTED.get(k, (0, 0))}
    assert not changed, changed
    missing = sorted(set(LISTED) - set(got))
    assert not missing, missing
