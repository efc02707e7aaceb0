"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the
CPU: the oracle (C, OpenMP) and the library's host-side query checks and
planning (C++), each built with gcc/g++ and the sanitizers into a small
driver that this test writes, run on seeded micro inputs, and compared
with the normal builds' answers. Any sanitizer report fails the run."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import paper_1807_08804_amd as P
from tests.micro import random_graph, random_query

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2")

ORACLE_DRIVER = r"""
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
typedef struct oracle_graph oracle_graph;
oracle_graph *oracle_graph_build(int32_t V, int64_t E, const int32_t *src, const int32_t *dst,
                                 const int32_t *rel, const int32_t *type);
void oracle_graph_free(oracle_graph *g);
int oracle_match(const oracle_graph *g, int32_t n, int32_t m, const int32_t *vlabel,
                 const int32_t *vpin, const int32_t *esrc, const int32_t *edst,
                 const int32_t *elabel, int64_t max_rows, int nthreads, int32_t **rows_out,
                 int64_t *nrows_out);
void oracle_free(void *p);
static int32_t rd(FILE *f) { int32_t x; if (fscanf(f, "%d", &x) != 1) exit(3); return x; }
int main(int argc, char **argv) {
    FILE *f = fopen(argv[1], "r");
    int32_t V = rd(f); int64_t E = rd(f);
    int32_t *s = malloc(4 * (E + 1)), *d = malloc(4 * (E + 1)), *r = malloc(4 * (E + 1));
    int32_t *t = malloc(4 * V);
    for (int64_t i = 0; i < E; ++i) { s[i] = rd(f); d[i] = rd(f); r[i] = rd(f); }
    for (int32_t v = 0; v < V; ++v) t[v] = rd(f);
    oracle_graph *g = oracle_graph_build(V, E, s, d, r, t);
    int32_t nq = rd(f);
    for (int32_t k = 0; k < nq; ++k) {
        int32_t n = rd(f), m = rd(f);
        int32_t vl[32], vp[32], es[64], ed[64], el[64];
        for (int u = 0; u < n; ++u) { vl[u] = rd(f); vp[u] = rd(f); }
        for (int e = 0; e < m; ++e) { es[e] = rd(f); ed[e] = rd(f); el[e] = rd(f); }
        int32_t *rows = NULL; int64_t nr = -1;
        int rc = oracle_match(g, n, m, vl, vp, es, ed, el, -1, 2, &rows, &nr);
        uint64_t h = 1469598103934665603ull;
        for (int64_t i = 0; rc == 0 && i < nr * n; ++i) h = (h ^ (uint32_t)rows[i]) * 1099511628211ull;
        printf("%d %lld %llu\n", rc, (long long)nr, (unsigned long long)h);
        oracle_free(rows);
    }
    oracle_graph_free(g);
    free(s); free(d); free(r); free(t);
    fclose(f);
    return 0;
}
"""

PLAN_DRIVER = r"""
#include <cstdio>
#include <cstdlib>
#include "sgm_plan.h"
using namespace sgm;
static int32_t rd(FILE *f) { int32_t x; if (std::fscanf(f, "%d", &x) != 1) std::exit(3); return x; }
int main(int argc, char **argv) {
    FILE *f = std::fopen(argv[1], "r");
    const int32_t V = rd(f);
    int64_t tf[8];
    for (int i = 0; i < 8; ++i) tf[i] = rd(f);
    int64_t rf[4];
    for (int i = 0; i < 4; ++i) rf[i] = rd(f);
    const int32_t nq = rd(f);
    for (int32_t k = 0; k < nq; ++k) {
        int32_t n = rd(f), m = rd(f);
        int32_t vl[SGM_MAX_QV], vp[SGM_MAX_QV], es[SGM_MAX_QE], ed[SGM_MAX_QE], el[SGM_MAX_QE];
        for (int u = 0; u < n; ++u) { vl[u] = rd(f); vp[u] = rd(f); }
        for (int e = 0; e < m; ++e) { es[e] = rd(f); ed[e] = rd(f); el[e] = rd(f); }
        sgm_query q{n, m, vl, vp, es, ed, el};
        QInfo qi;
        int rc = check_query(&q, V, &qi);
        if (rc) { std::printf("%d\n", rc); continue; }
        Plan pl;
        rc = make_plan(qi, V, tf, 8, &pl);
        Program a, b;
        build_program(qi, pl, 1, 1, &a);
        build_program_out_only(qi, pl, 1, 1, &b);
        const int64_t est = estimate_bytes(qi, pl, V, 4 * V, tf, 8, rf, 4);
        int ok = set_projection(&qi, 1u);
        std::printf("%d %d", rc, ok);
        for (int i = 0; i < pl.n_visit; ++i) std::printf(" %d", pl.visit[i]);
        std::printf(" | %d %d %d %d %d %d %lld\n", a.init.size(), a.refine.size(), a.nbr.size(),
                    b.init.size(), b.refine.size(), b.nbr.size(), (long long)est);
    }
    std::fclose(f);
    return 0;
}
"""


COMPRESS_DRIVER = r"""
#include <cstdio>
#include <cstdlib>
#include "sgm.h"
static int32_t rd(FILE *f) { int32_t x; if (std::fscanf(f, "%d", &x) != 1) std::exit(3); return x; }
int main(int argc, char **argv) {
    FILE *f = std::fopen(argv[1], "r");
    const int32_t V = rd(f), E = rd(f);
    int32_t *rp = new int32_t[V + 1], *col = new int32_t[E + 1], *rel = new int32_t[E + 1];
    int32_t *typ = new int32_t[V];
    for (int32_t v = 0; v <= V; ++v) rp[v] = rd(f);
    for (int32_t i = 0; i < E; ++i) { col[i] = rd(f); rel[i] = rd(f); }
    for (int32_t v = 0; v < V; ++v) typ[v] = rd(f);
    const int32_t nd = rd(f);
    for (int k = 0; k < nd; ++k) {
        sgm_compress_options o;
        sgm_default_compress_options(&o);
        o.max_levels = 4;
        for (int i = 0; i < 8; ++i) o.delta[i] = rd(f) / 100.0f;
        sgm_compressed *c = nullptr;
        const int rc = sgm_compress(V, E, rp, col, rel, typ, &o, &c);
        unsigned long long h = 1469598103934665603ull;
        auto mix = [&](const int32_t *a, int64_t n) {
            for (int64_t i = 0; i < n; ++i) h = (h ^ (uint32_t)a[i]) * 1099511628211ull;
        };
        if (rc == 0) {
            mix(c->row_ptr, c->n_vertices + 1); mix(c->col, c->n_edges); mix(c->rel, c->n_edges);
            mix(c->weight, c->n_edges); mix(c->out_bound, c->n_vertices); mix(c->in_bound, c->n_vertices);
            mix(c->map_off, c->n_vertices + 1); mix(c->map_ids, V); mix(c->hyper_of, V);
            std::printf("%d %d %lld %llu\n", rc, c->n_vertices, (long long)c->n_edges, h);
        } else {
            std::printf("%d\n", rc);
        }
        sgm_free_compressed(c);
    }
    delete[] rp; delete[] col; delete[] rel; delete[] typ;
    std::fclose(f);
    return 0;
}
"""


def _compile(tool, args, tmp_path):
    exe = str(tmp_path / "drv")
    p = subprocess.run([tool, *SAN, *args, "-o", exe], capture_output=True, text=True)
    if p.returncode != 0:
        pytest.fail(p.stdout + p.stderr)
    return exe


def _run(exe, inp):
    p = subprocess.run([exe, str(inp)], capture_output=True, text=True, env=ENV, timeout=300)
    assert p.returncode == 0 and "runtime error" not in p.stderr and \
        "AddressSanitizer" not in p.stderr, p.stderr[-4000:]
    return p.stdout.split("\n")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc is not installed")
def test_oracle_under_sanitizers(tmp_path):
    rng = np.random.default_rng(404)
    lines, cases = [], []
    mg = random_graph(rng, 40, 160, n_types=3, n_rels=3)
    lines.append(f"{mg.V} {len(mg.src)}")
    lines += [f"{a} {b} {r}" for a, b, r in zip(mg.src, mg.dst, mg.rel)]
    lines.append(" ".join(str(int(t)) for t in mg.vtype))
    qs = [random_query(rng, int(rng.integers(1, 7)), 3, 3, mg.V, p_pin=0.2, extra=3)
          for _ in range(40)]
    lines.append(str(len(qs)))
    for q in qs:
        lines.append(f"{q.n} {q.m}")
        lines += [f"{int(a)} {int(b)}" for a, b in zip(q.vlabel, q.vpin)]
        lines += [f"{int(a)} {int(b)} {int(c)}" for a, b, c in zip(q.esrc, q.edst, q.elabel)]
    inp = tmp_path / "in.txt"
    inp.write_text("\n".join(lines) + "\n")
    src = tmp_path / "drv.c"
    src.write_text(ORACLE_DRIVER)
    exe = _compile("gcc", ["-fopenmp", str(src), os.path.join(ROOT, "oracle", "sgm_oracle.c")],
                   tmp_path)
    out = _run(exe, inp)
    og = oracle.Graph(mg.V, mg.src, mg.dst, mg.rel, mg.vtype)
    for q, line in zip(qs, out):
        rc, nr, h = line.split()
        want = og.match_query(q)
        assert int(rc) == 0 and int(nr) == len(want), (q, line)
        hh = 1469598103934665603
        for x in want.reshape(-1).astype(np.uint32).tolist():
            hh = ((hh ^ x) * 1099511628211) & ((1 << 64) - 1)
        assert int(h) == hh, q


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ is not installed")
def test_host_planning_under_sanitizers(tmp_path):
    rng = np.random.default_rng(405)
    V = 1000
    tf = rng.integers(1, 300, 8)
    rf = rng.integers(1, 2000, 4)
    qs = [random_query(rng, int(rng.integers(1, 17)), 8, 4, V, p_pin=0.2, extra=6)
          for _ in range(200)]
    lines = [str(V), " ".join(map(str, tf)), " ".join(map(str, rf)), str(len(qs))]
    for q in qs:
        lines.append(f"{q.n} {q.m}")
        lines += [f"{int(a)} {int(b)}" for a, b in zip(q.vlabel, q.vpin)]
        lines += [f"{int(a)} {int(b)} {int(c)}" for a, b, c in zip(q.esrc, q.edst, q.elabel)]
    inp = tmp_path / "in.txt"
    inp.write_text("\n".join(lines) + "\n")
    src = tmp_path / "drv.cpp"
    src.write_text(PLAN_DRIVER)
    csrc = os.path.join(ROOT, "paper_1807_08804_amd", "csrc")
    exe = _compile("g++", ["-std=c++17", "-I", csrc, str(src), os.path.join(csrc, "sgm_plan.cpp")],
                   tmp_path)
    out = _run(exe, inp)
    for q, line in zip(qs, out):
        if line.split()[0] != "0":
            continue
        visit = [int(x) for x in line.split("|")[0].split()[2:]]
        p = P.sgm_plan_query(q.n, q.vlabel, q.vpin, q.esrc, q.edst, q.elabel, V, tf)
        assert visit == p["visit_order"], (q, line)


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ is not installed")
def test_compression_under_sanitizers(tmp_path):
    """sgm_compress (host code) built with the sanitizers on micro graphs
    with repeated triples and self-loops at several thresholds: no report,
    and the same weighted graph and mapping as the library's build."""
    rng = np.random.default_rng(406)
    mg = random_graph(rng, 80, 400, n_types=2, n_rels=3)
    rp, col, rel, typ = mg.csr()
    deltas = [[100] * 8, [50] * 8, [20] * 8]
    lines = [f"{len(rp) - 1} {len(col)}", " ".join(map(str, rp))]
    lines += [f"{int(a)} {int(b)}" for a, b in zip(col, rel)]
    lines += [" ".join(map(str, typ)), str(len(deltas))] + [" ".join(map(str, d)) for d in deltas]
    inp = tmp_path / "in.txt"
    inp.write_text("\n".join(lines) + "\n")
    src = tmp_path / "drv.cpp"
    src.write_text(COMPRESS_DRIVER)
    csrc = os.path.join(ROOT, "paper_1807_08804_amd", "csrc")
    exe = _compile("g++", ["-std=c++17", "-I", os.path.join(ROOT, "include"), str(src),
                           os.path.join(csrc, "sgm_compress.cpp")], tmp_path)
    out = _run(exe, inp)
    for d, line in zip(deltas, out):
        c = P.Compressed(rp, col, rel, typ, max_levels=4, delta=d[0] / 100.0)
        h = 1469598103934665603
        for a in (c.row_ptr, c.col, c.rel, c.weight, c.out_bound, c.in_bound, c.map_off,
                  c.map_ids, c.hyper_of):
            for x in a.astype(np.uint32).tolist():
                h = ((h ^ x) * 1099511628211) & ((1 << 64) - 1)
        assert line.split() == ["0", str(c.n_vertices), str(c.n_edges), str(h)], (d, line)
