"""CPU checks of the Python binding's classes, read from their source: every
``self.<name>`` a method of Plan, Batch or Fourier reads is defined by that
class (a method, a property, a class attribute or an attribute assigned in
one of its methods), so no method copied from one class into another can
reach for attributes that only the other holds."""
import ast
import inspect

import pytest

from paper_2006_01573_amd import ctis


def _defined_and_used(cls):
    tree = ast.parse(inspect.getsource(cls))
    node = tree.body[0]
    assert isinstance(node, ast.ClassDef)
    defined, used = set(), {}
    for item in node.body:
        if isinstance(item, (ast.FunctionDef, ast.AsyncFunctionDef)):
            defined.add(item.name)
        elif isinstance(item, ast.Assign):
            defined.update(t.id for t in item.targets if isinstance(t, ast.Name))
        elif isinstance(item, ast.AnnAssign) and isinstance(item.target, ast.Name):
            defined.add(item.target.id)
    for item in node.body:
        if not isinstance(item, ast.FunctionDef):
            continue
        for sub in ast.walk(item):
            if isinstance(sub, ast.Attribute) and isinstance(sub.value, ast.Name) and sub.value.id == "self":
                if isinstance(sub.ctx, ast.Store):
                    defined.add(sub.attr)
                else:
                    used.setdefault(sub.attr, item.name)
    return defined, used


@pytest.mark.parametrize("cls", [ctis.Plan, ctis.Batch, ctis.Fourier], ids=lambda c: c.__name__)
def test_methods_read_only_their_own_attributes(cls):
    defined, used = _defined_and_used(cls)
    inherited = {n for n in dir(object)}
    missing = {a: m for a, m in used.items() if a not in defined and a not in inherited}
    assert not missing, f"{cls.__name__} methods read attributes it never defines: {missing}"


def test_plan_only_calls_are_not_on_batches():
    # the C ABI has no batch forms of the diagnostics or the scratch-free EM
    assert hasattr(ctis.Plan, "diagnostics") and hasattr(ctis.Plan, "em_static")
    assert not hasattr(ctis.Batch, "diagnostics") and not hasattr(ctis.Batch, "em_static")
