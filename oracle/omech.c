/*
 * Oracle mechanism parser (test infrastructure; see oracle.h).
 * Reads the plain-text mechanism format, converts CHEMKIN units
 * (cm, mol, s, cal/mol, g/mol) to SI.
 */
#include "oracle.h"

#include <ctype.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    char **tok;
    int n, pos;
    char *buf;
} tokens_t;

static int tokenize(const char *path, tokens_t *tk) {
    FILE *f = fopen(path, "rb");
    if (!f) return -1;
    fseek(f, 0, SEEK_END);
    long len = ftell(f);
    fseek(f, 0, SEEK_SET);
    tk->buf = (char *)malloc(len + 1);
    if (fread(tk->buf, 1, len, f) != (size_t)len) {
        fclose(f);
        return -1;
    }
    tk->buf[len] = 0;
    fclose(f);
    /* blank out comments */
    for (long i = 0; i < len; i++) {
        if (tk->buf[i] == '#') {
            while (i < len && tk->buf[i] != '\n') tk->buf[i++] = ' ';
        }
    }
    int cap = 1024;
    tk->tok = (char **)malloc(cap * sizeof(char *));
    tk->n = 0;
    tk->pos = 0;
    char *p = tk->buf;
    while (*p) {
        while (*p && isspace((unsigned char)*p)) p++;
        if (!*p) break;
        if (tk->n == cap) {
            cap *= 2;
            tk->tok = (char **)realloc(tk->tok, cap * sizeof(char *));
        }
        tk->tok[tk->n++] = p;
        while (*p && !isspace((unsigned char)*p)) p++;
        if (*p) *p++ = 0;
    }
    return 0;
}

static const char *next(tokens_t *tk) { return tk->pos < tk->n ? tk->tok[tk->pos++] : NULL; }
static const char *peek(tokens_t *tk) { return tk->pos < tk->n ? tk->tok[tk->pos] : NULL; }

static int expect(tokens_t *tk, const char *kw) {
    const char *t = next(tk);
    return t && strcmp(t, kw) == 0;
}

static int get_int(tokens_t *tk, int *v) {
    const char *t = next(tk);
    if (!t) return 0;
    char *end;
    long x = strtol(t, &end, 10);
    if (*end) return 0;
    *v = (int)x;
    return 1;
}

static int get_dbl(tokens_t *tk, double *v) {
    const char *t = next(tk);
    if (!t) return 0;
    char *end;
    *v = strtod(t, &end);
    return *end == 0;
}

static int find_sp(const omech_t *m, const char *name) {
    for (int k = 0; k < m->ns; k++)
        if (strcmp(m->sp[k], name) == 0) return k;
    return -1;
}

#define FAIL(msg)                                                   \
    do {                                                            \
        snprintf(err, errlen, "%s (token %d)", msg, tk.pos);       \
        goto fail;                                                  \
    } while (0)

int omech_load(const char *path, omech_t **out, char *err, int errlen) {
    tokens_t tk = {0};
    omech_t *m = (omech_t *)calloc(1, sizeof(omech_t));
    if (tokenize(path, &tk) != 0) {
        snprintf(err, errlen, "cannot read %s", path);
        free(m);
        return -1;
    }
    if (!expect(&tk, "MECHANISM")) FAIL("expected MECHANISM");
    {
        const char *nm = next(&tk);
        if (!nm) FAIL("missing name");
        snprintf(m->name, sizeof m->name, "%s", nm);
    }
    if (!expect(&tk, "UNITS") || !expect(&tk, "CM-MOL-S") || !expect(&tk, "CAL/MOL"))
        FAIL("expected UNITS CM-MOL-S CAL/MOL");
    if (!expect(&tk, "ELEMENTS") || !get_int(&tk, &m->ne) || m->ne <= 0) FAIL("bad ELEMENTS");
    m->elem = calloc(m->ne, sizeof *m->elem);
    for (int i = 0; i < m->ne; i++) {
        const char *e = next(&tk);
        if (!e) FAIL("bad element");
        snprintf(m->elem[i], 8, "%s", e);
    }
    if (!expect(&tk, "SPECIES") || !get_int(&tk, &m->ns) || m->ns <= 0) FAIL("bad SPECIES");
    int ns = m->ns;
    m->sp = calloc(ns, sizeof *m->sp);
    m->W = calloc(ns, sizeof(double));
    m->comp = calloc((size_t)ns * m->ne, sizeof(int));
    for (int k = 0; k < ns; k++) {
        const char *nm = next(&tk);
        if (!nm) FAIL("bad species");
        snprintf(m->sp[k], 32, "%s", nm);
        double w;
        if (!get_dbl(&tk, &w) || w <= 0) FAIL("bad molecular weight");
        m->W[k] = w * 1e-3;
        for (int e = 0; e < m->ne; e++)
            if (!get_int(&tk, &m->comp[k * m->ne + e])) FAIL("bad composition");
    }
    for (int k = 0; k < ns; k++)
        for (int j = 0; j < k; j++)
            if (strcmp(m->sp[k], m->sp[j]) == 0) FAIL("duplicate species");
    if (!expect(&tk, "THERMO")) FAIL("expected THERMO");
    m->Tlo = calloc(ns, sizeof(double));
    m->Tmid = calloc(ns, sizeof(double));
    m->Thi = calloc(ns, sizeof(double));
    m->alo = calloc(ns * 7, sizeof(double));
    m->ahi = calloc(ns * 7, sizeof(double));
    {
        int *seen = calloc(ns, sizeof(int));
        for (int i = 0; i < ns; i++) {
            const char *nm = next(&tk);
            int k = nm ? find_sp(m, nm) : -1;
            if (k < 0 || seen[k]) {
                free(seen);
                FAIL("bad THERMO species");
            }
            seen[k] = 1;
            if (!get_dbl(&tk, &m->Tlo[k]) || !get_dbl(&tk, &m->Tmid[k]) || !get_dbl(&tk, &m->Thi[k])) {
                free(seen);
                FAIL("bad THERMO range");
            }
            for (int a = 0; a < 7; a++)
                if (!get_dbl(&tk, &m->alo[k * 7 + a])) {
                    free(seen);
                    FAIL("bad NASA coefficient");
                }
            for (int a = 0; a < 7; a++)
                if (!get_dbl(&tk, &m->ahi[k * 7 + a])) {
                    free(seen);
                    FAIL("bad NASA coefficient");
                }
        }
        free(seen);
    }
    if (!expect(&tk, "REACTIONS") || !get_int(&tk, &m->nr) || m->nr < 0) FAIL("bad REACTIONS");
    int nr = m->nr;
    int nrr = nr > 0 ? nr : 1;
    m->type = calloc(nrr, sizeof(int));
    m->rev = calloc(nrr, sizeof(int));
    m->nre = calloc(nrr, sizeof(int));
    m->npr = calloc(nrr, sizeof(int));
    m->rsp = calloc(nrr * OR_MAXPART, sizeof(int));
    m->rnu = calloc(nrr * OR_MAXPART, sizeof(int));
    m->psp = calloc(nrr * OR_MAXPART, sizeof(int));
    m->pnu = calloc(nrr * OR_MAXPART, sizeof(int));
    m->A = calloc(nrr, sizeof(double));
    m->b = calloc(nrr, sizeof(double));
    m->Ea = calloc(nrr, sizeof(double));
    m->eff = calloc((size_t)nrr * ns, sizeof(double));
    m->A0 = calloc(nrr, sizeof(double));
    m->b0 = calloc(nrr, sizeof(double));
    m->Ea0 = calloc(nrr, sizeof(double));
    m->troe_n = calloc(nrr, sizeof(int));
    m->troe = calloc(nrr * 4, sizeof(double));
    for (int j = 0; j < nr; j++) {
        if (!expect(&tk, "REACTION")) FAIL("expected REACTION");
        const char *ty = next(&tk), *rv = next(&tk);
        if (!ty || !rv) FAIL("bad REACTION header");
        if (!strcmp(ty, "ELEMENTARY")) m->type[j] = OR_ELEM;
        else if (!strcmp(ty, "THREEBODY")) m->type[j] = OR_THREEBODY;
        else if (!strcmp(ty, "FALLOFF")) m->type[j] = OR_FALLOFF;
        else FAIL("unknown reaction type");
        if (!strcmp(rv, "REV")) m->rev[j] = 1;
        else if (!strcmp(rv, "IRREV")) m->rev[j] = 0;
        else FAIL("expected REV or IRREV");
        for (int k = 0; k < ns; k++) m->eff[(size_t)j * ns + k] = 1.0;
        int have_arr = 0, have_low = 0;
        int have_side[2] = {0, 0};
        for (;;) {
            const char *kw = next(&tk);
            if (!kw) FAIL("unterminated REACTION");
            if (!strcmp(kw, "END")) break;
            if (!strcmp(kw, "REACTANTS") || !strcmp(kw, "PRODUCTS")) {
                int isr = kw[0] == 'R';
                int cnt;
                if (!get_int(&tk, &cnt) || cnt <= 0 || cnt > OR_MAXPART) FAIL("bad participant count");
                for (int i = 0; i < cnt; i++) {
                    const char *nm = next(&tk);
                    int k = nm ? find_sp(m, nm) : -1, nu;
                    if (k < 0) FAIL("unknown species in reaction");
                    if (!get_int(&tk, &nu) || nu <= 0 || nu > 3) FAIL("bad stoichiometric coefficient");
                    for (int q = 0; q < i; q++)
                        if ((isr ? m->rsp : m->psp)[j * OR_MAXPART + q] == k) FAIL("repeated species on one side");
                    if (isr) {
                        m->rsp[j * OR_MAXPART + i] = k;
                        m->rnu[j * OR_MAXPART + i] = nu;
                    } else {
                        m->psp[j * OR_MAXPART + i] = k;
                        m->pnu[j * OR_MAXPART + i] = nu;
                    }
                }
                if (isr) m->nre[j] = cnt;
                else m->npr[j] = cnt;
                have_side[isr ? 0 : 1] = 1;
            } else if (!strcmp(kw, "ARRHENIUS")) {
                if (!get_dbl(&tk, &m->A[j]) || !get_dbl(&tk, &m->b[j]) || !get_dbl(&tk, &m->Ea[j]))
                    FAIL("bad ARRHENIUS");
                have_arr = 1;
            } else if (!strcmp(kw, "EFFICIENCIES")) {
                int cnt;
                if (!get_int(&tk, &cnt) || cnt < 0) FAIL("bad EFFICIENCIES");
                for (int i = 0; i < cnt; i++) {
                    const char *nm = next(&tk);
                    int k = nm ? find_sp(m, nm) : -1;
                    double a;
                    if (!get_dbl(&tk, &a)) FAIL("bad efficiency");
                    if (k >= 0) m->eff[(size_t)j * ns + k] = a; /* absent species ignored */
                }
            } else if (!strcmp(kw, "LOW")) {
                if (!get_dbl(&tk, &m->A0[j]) || !get_dbl(&tk, &m->b0[j]) || !get_dbl(&tk, &m->Ea0[j]))
                    FAIL("bad LOW");
                have_low = 1;
            } else if (!strcmp(kw, "TROE")) {
                int cnt;
                if (!get_int(&tk, &cnt) || (cnt != 3 && cnt != 4)) FAIL("bad TROE count");
                m->troe_n[j] = cnt;
                for (int i = 0; i < cnt; i++)
                    if (!get_dbl(&tk, &m->troe[j * 4 + i])) FAIL("bad TROE parameter");
            } else {
                FAIL("unknown reaction keyword");
            }
        }
        if (!have_arr || !have_side[0] || !have_side[1]) FAIL("incomplete reaction");
        if (m->type[j] == OR_FALLOFF && !have_low) FAIL("FALLOFF without LOW");
        /* element balance */
        for (int e = 0; e < m->ne; e++) {
            long bal = 0;
            for (int i = 0; i < m->nre[j]; i++)
                bal -= (long)m->rnu[j * OR_MAXPART + i] * m->comp[m->rsp[j * OR_MAXPART + i] * m->ne + e];
            for (int i = 0; i < m->npr[j]; i++)
                bal += (long)m->pnu[j * OR_MAXPART + i] * m->comp[m->psp[j * OR_MAXPART + i] * m->ne + e];
            if (bal != 0) FAIL("reaction not element-balanced");
        }
        /* CHEMKIN -> SI: (cm^3/mol)^(order-1) -> (m^3/mol)^(order-1) */
        int order = 0;
        for (int i = 0; i < m->nre[j]; i++) order += m->rnu[j * OR_MAXPART + i];
        int order_inf = order + (m->type[j] == OR_THREEBODY ? 1 : 0);
        m->A[j] *= pow(1e-6, order_inf - 1);
        m->Ea[j] *= OR_CAL;
        if (m->type[j] == OR_FALLOFF) {
            m->A0[j] *= pow(1e-6, order);
            m->Ea0[j] *= OR_CAL;
        }
    }
    if (!expect(&tk, "END")) FAIL("expected END");
    free(tk.tok);
    free(tk.buf);
    *out = m;
    return 0;
fail:
    free(tk.tok);
    free(tk.buf);
    omech_free(m);
    return -1;
}

void omech_free(omech_t *m) {
    if (!m) return;
    free(m->elem); free(m->sp); free(m->W); free(m->comp);
    free(m->Tlo); free(m->Tmid); free(m->Thi); free(m->alo); free(m->ahi);
    free(m->type); free(m->rev); free(m->nre); free(m->npr);
    free(m->rsp); free(m->rnu); free(m->psp); free(m->pnu);
    free(m->A); free(m->b); free(m->Ea); free(m->eff);
    free(m->A0); free(m->b0); free(m->Ea0); free(m->troe_n); free(m->troe);
    free(m);
}
