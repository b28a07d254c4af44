"""Every name a function of the repository's Python files reads is defined in
that function, an enclosing one, its module or the builtins. GPU-only tests
never run on the CPU, so a misspelt or misplaced variable in one would otherwise
surface only on a GPU."""
import ast
import builtins
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FILES = sorted(
    [os.path.join("tests", f) for f in os.listdir(os.path.join(ROOT, "tests")) if f.endswith(".py")]
    + [os.path.join("paper_2108_12240_amd", f) for f in os.listdir(os.path.join(ROOT, "paper_2108_12240_amd"))
       if f.endswith(".py")]
    + [os.path.join("oracle", f) for f in os.listdir(os.path.join(ROOT, "oracle")) if f.endswith(".py")]
    + ["bench.py", "__graft_entry__.py"])


def bound_names(node):
    """Names a scope binds: arguments, assignment and loop targets, imports,
    nested definitions, with/except aliases, comprehension variables."""
    out = set()
    if isinstance(node, (ast.FunctionDef, ast.AsyncFunctionDef, ast.Lambda)):
        a = node.args
        for arg in a.posonlyargs + a.args + a.kwonlyargs + [a.vararg, a.kwarg]:
            if arg is not None:
                out.add(arg.arg)
    body = node.body if isinstance(node.body, list) else [node.body]
    stack = list(body)
    while stack:
        n = stack.pop()
        if isinstance(n, (ast.FunctionDef, ast.AsyncFunctionDef, ast.ClassDef)):
            out.add(n.name)
            out.update(d.id for d in n.decorator_list if isinstance(d, ast.Name))
            continue                                   # its own scope
        if isinstance(n, ast.Lambda):
            continue
        if isinstance(n, ast.Name) and isinstance(n.ctx, (ast.Store, ast.Del)):
            out.add(n.id)
        elif isinstance(n, (ast.Import, ast.ImportFrom)):
            out.update((al.asname or al.name).split(".")[0] for al in n.names)
        elif isinstance(n, ast.ExceptHandler) and n.name:
            out.add(n.name)
        elif isinstance(n, (ast.Global, ast.Nonlocal)):
            out.update(n.names)
        stack.extend(ast.iter_child_nodes(n))
    return out


def undefined(tree):
    missing = []
    builtin = set(dir(builtins)) | {"__file__", "__name__", "__doc__"}

    def visit(node, visible):
        scope = visible | bound_names(node)
        body = node.body if isinstance(node.body, list) else [node.body]
        stack = list(body)
        if isinstance(node, (ast.FunctionDef, ast.AsyncFunctionDef, ast.Lambda)):
            stack += [d for d in node.args.defaults + node.args.kw_defaults if d is not None]
        while stack:
            n = stack.pop()
            if isinstance(n, (ast.FunctionDef, ast.AsyncFunctionDef, ast.Lambda)):
                visit(n, scope)
                continue
            if isinstance(n, ast.ClassDef):
                visit(n, scope)
                continue
            if isinstance(n, ast.Name) and isinstance(n.ctx, ast.Load) and n.id not in scope | builtin:
                missing.append((n.id, n.lineno))
            stack.extend(ast.iter_child_nodes(n))

    visit(tree, set())
    return missing


@pytest.mark.parametrize("path", FILES)
def test_no_undefined_names(path):
    with open(os.path.join(ROOT, path), encoding="utf-8") as f:
        tree = ast.parse(f.read(), path)
    assert undefined(tree) == [], path


def test_the_check_finds_a_misplaced_name():
    src = "def f(a):\n    return a + b\n\ndef g():\n    fused = 1\n    return fused\n"
    assert undefined(ast.parse(src)) == [("b", 2)]
    src2 = "import numpy as np\nX = [i for i in range(3)]\ndef h(q=np.pi):\n    return [j * q for j in X]\n"
    assert undefined(ast.parse(src2)) == []
