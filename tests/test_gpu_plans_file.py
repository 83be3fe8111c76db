"""Saving and loading the autotuners' plans (fla_save_plans, fla_load_plans):
a round trip through a file, lines for another architecture ignored, and a
malformed file rejected without changing anything."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import paper_2512_20829_amd as F
    return F


def test_plans_round_trip(F, tmp_path):
    a, b = F.Context(0), F.Context(0)
    try:
        a.set_plan(3, F.FLA_F32, 5)
        a.set_plan(2, F.FLA_F64, 2)
        a.set_batch_plan(3, F.FLA_F32, 4, 64)
        path = tmp_path / "plans.txt"
        a.save_plans(str(path))
        text = path.read_text().splitlines()
        assert text[0] == "flaproj-plans 1" and len(text) == 5
        arch = text[1].split()[0]
        assert arch.startswith("gfx")
        b.load_plans(str(path))
        assert b.get_plan(3, F.FLA_F32) == 5 and b.get_plan(2, F.FLA_F64) == 2
        assert b.get_batch_plan(3, F.FLA_F32) == (4, 64)
        assert b.get_plan(3, F.FLA_F64) == 1          # -1 in the file: the default stays
        # lines for another architecture are ignored
        other = tmp_path / "other.txt"
        other.write_text("flaproj-plans 1\ngfx000 3 0 7 7 4\n")
        b.load_plans(str(other))
        assert b.get_plan(3, F.FLA_F32) == 5
    finally:
        a.close()
        b.close()


@pytest.mark.parametrize("bad_line", [None, "{arch} 3 0 9 -1 16", "{arch} 2 0 4 -1 16", "{arch} 3 0 1 1 0",
                                      "{arch} 3 0 1"])
def test_bad_plan_files_change_nothing(F, tmp_path, bad_line):
    """No header, a plan code beyond the dimension's, a batch chunk of 0, a
    short line: INVALID_ARG, and the valid line before it is not applied."""
    c = F.Context(0)
    try:
        good = tmp_path / "good.txt"
        c.save_plans(str(good))
        arch = good.read_text().splitlines()[1].split()[0]
        c.set_plan(3, F.FLA_F32, 6)
        bad = tmp_path / "bad.txt"
        if bad_line is None:
            bad.write_text(f"not a plan file\n{arch} 3 1 2 -1 16\n")
        else:
            bad.write_text(f"flaproj-plans 1\n{arch} 3 1 2 -1 16\n" + bad_line.format(arch=arch) + "\n")
        with pytest.raises(F.FlaError, match="INVALID_ARG"):
            c.load_plans(str(bad))
        assert c.get_plan(3, F.FLA_F32) == 6 and c.get_plan(3, F.FLA_F64) == 1
        with pytest.raises(F.FlaError, match="INVALID_ARG"):
            c.load_plans(str(tmp_path / "missing.txt"))
    finally:
        c.close()
