"""The build script's unit tables name real sources: the per-unit code-generation
flags and the slow-first compile order would otherwise drop silently when a
unit is renamed or split."""
import os

from paper_1909_11474_amd import build as B


def test_unit_tables_name_existing_sources():
    names = {os.path.basename(p) for p in B.sources()}
    assert set(B.UNIT_FLAGS) <= names, sorted(set(B.UNIT_FLAGS) - names)
    assert set(B.SLOW_UNITS) <= names, sorted(set(B.SLOW_UNITS) - names)


def test_slow_units_start_first_and_every_unit_is_built():
    order = [os.path.basename(p) for p in B._build_order(B.sources())]
    assert order[:len(B.SLOW_UNITS)] == list(B.SLOW_UNITS)
    assert sorted(order) == sorted(os.path.basename(p) for p in B.sources())


def test_unit_flags_are_compiler_options_only():
    for unit, flags in B.UNIT_FLAGS.items():
        assert flags and all(f.startswith("-") for f in flags), unit
        assert not any(f.startswith("-fsanitize") for f in flags), unit
