"""The build entry point in a checkout with no built library: the build
module loads without the library, reports it stale, and the package itself
refuses to import (no fallback). Also: a source newer than the library
marks it stale, and ensure_built() rebuilds exactly then."""
import os
import shutil
import subprocess
import sys
import textwrap

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _fresh_tree(tmp_path):
    dst = tmp_path / "repo"
    ign = shutil.ignore_patterns("*.so", "*.so.tmp", "__pycache__", "*.o")
    for d in ("paper_1401_5245_amd", "include", "oracle", "synth"):
        shutil.copytree(os.path.join(ROOT, d), dst / d, ignore=ign)
    shutil.copy(os.path.join(ROOT, "__graft_entry__.py"), dst / "__graft_entry__.py")
    return dst


def _run(tree, code):
    return subprocess.run([sys.executable, "-c", textwrap.dedent(code)], cwd=tree,
                          capture_output=True, text=True, timeout=300)


def test_build_module_loads_without_library(tmp_path):
    tree = _fresh_tree(tmp_path)
    assert not (tree / "paper_1401_5245_amd" / "libedgemask.so").exists()
    r = _run(tree, """
        import __graft_entry__ as g
        m = g._hip_build_module()
        assert m.is_stale()
        srcs = m.units()
        assert len(srcs) >= 2, srcs
        for s in srcs:
            cmd = m.compile_command(s, "x.o")
            assert "--offload-arch=gfx950" in cmd
            i = cmd.index("-packed-fp32-ops")
            assert cmd[i - 1] == "-Xclang" and cmd[i - 2] == "-target-feature"
        try:
            import paper_1401_5245_amd
        except ImportError as e:
            assert "not built" in str(e), e
            print("REFUSED")
    """)
    assert r.returncode == 0, r.stderr
    assert "REFUSED" in r.stdout


def test_ensure_built_rebuilds_only_when_stale(tmp_path):
    tree = _fresh_tree(tmp_path)
    lib = tree / "paper_1401_5245_amd" / "libedgemask.so"
    r = _run(tree, """
        import os, time
        import __graft_entry__ as g
        calls = []
        g.build = lambda: calls.append(1)
        g.ensure_built()                      # no library: builds
        assert calls == [1], calls
        lib = os.path.join("paper_1401_5245_amd", "libedgemask.so")
        open(lib, "wb").close()
        future = time.time() + 100
        os.utime(lib, (future, future))
        g.ensure_built()                      # newer than every source: nothing
        assert calls == [1], calls
        src = os.path.join("paper_1401_5245_amd", "csrc", "edge_masks.hip")
        os.utime(src, (future + 50, future + 50))
        g.ensure_built()                      # a source changed: builds again
        assert calls == [1, 1], calls
        print("OK")
    """)
    assert r.returncode == 0, r.stderr
    assert "OK" in r.stdout
    assert lib.exists()
