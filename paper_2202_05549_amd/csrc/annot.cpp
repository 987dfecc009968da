// Annotation compiler: data-access annotation text -> affine index forms.
//
// Grammar (Sec. 2.3 "Data Annotations"):
//   annotation := binding { ',' binding } '=>' access { ',' access }
//   binding    := ('global' | 'block' | 'local') names
//   names      := IDENT | '[' IDENT { ',' IDENT } ']'     (slowest axis first)
//   access     := mode IDENT '[' index { ',' index } ']'
//   mode       := 'read' | 'write' | 'readwrite' | 'reduce' '(' op ')'
//   op         := '+' | '*' | 'min' | 'max'
//   index      := expr | [expr] ':' [expr]                 (inclusive slice)
//   expr       := linear combination of bound variables, integer literals and
//                 integer scalar parameters of the kernel, with + - * ( ).
// A product of two non-constant terms is rejected (indices must be linear in
// the bound variables); so is any name that is neither bound nor an integer
// parameter, which also rules out indirection such as A[B[i]] (Sec. 2.5).
#include <cctype>
#include <cstdarg>
#include <cstdio>

#include "lt_internal.h"

namespace lt {

namespace {

struct Tok {
    enum K { END, IDENT, NUM, SYM } k;
    std::string s;
    int64_t v = 0;
    size_t pos = 0;
};

struct Lexer {
    const std::string &t;
    size_t i = 0;
    explicit Lexer(const std::string &text) : t(text) {}
    bool next(Tok *out, std::string *err) {
        while (i < t.size() && isspace((unsigned char)t[i])) ++i;
        out->pos = i;
        if (i >= t.size()) {
            out->k = Tok::END;
            out->s.clear();
            return true;
        }
        char c = t[i];
        if (isalpha((unsigned char)c) || c == '_') {
            size_t j = i;
            while (j < t.size() && (isalnum((unsigned char)t[j]) || t[j] == '_')) ++j;
            out->k = Tok::IDENT;
            out->s = t.substr(i, j - i);
            i = j;
            return true;
        }
        if (isdigit((unsigned char)c)) {
            size_t j = i;
            int64_t v = 0;
            while (j < t.size() && isdigit((unsigned char)t[j])) {
                if (v > (INT64_MAX - 9) / 10) {
                    *err = "integer literal too large";
                    return false;
                }
                v = v * 10 + (t[j] - '0');
                ++j;
            }
            out->k = Tok::NUM;
            out->v = v;
            out->s = t.substr(i, j - i);
            i = j;
            return true;
        }
        if (c == '=' && i + 1 < t.size() && t[i + 1] == '>') {
            out->k = Tok::SYM;
            out->s = "=>";
            i += 2;
            return true;
        }
        if (strchr("[](),:+-*", c)) {
            out->k = Tok::SYM;
            out->s = std::string(1, c);
            ++i;
            return true;
        }
        char buf[64];
        snprintf(buf, sizeof buf, "unexpected character '%c' at %zu", c, i);
        *err = buf;
        return false;
    }
};

struct Parser {
    const KernelDef *def;
    std::vector<Tok> toks;
    size_t k = 0;
    std::string err;
    // bound name -> variable slot
    std::vector<std::pair<std::string, int>> vars;

    const Tok &peek() const { return toks[k]; }
    bool is(const char *sym) const {
        return (peek().k == Tok::SYM || peek().k == Tok::IDENT) && peek().s == sym;
    }
    bool fail(const std::string &m) {
        if (err.empty()) {
            char buf[48];
            snprintf(buf, sizeof buf, " (at offset %zu)", peek().pos);
            err = m + buf;
        }
        return false;
    }
    bool expect(const char *sym) {
        if (!is(sym)) return fail(std::string("expected '") + sym + "', found '" + peek().s + "'");
        ++k;
        return true;
    }

    int find_param(const std::string &n, int kind) const {
        for (int p = 0; p < def->nparam; ++p)
            if (n == def->params[p].name && (kind < 0 || def->params[p].kind == kind)) return p;
        return -1;
    }

    bool primary(Affine *out) {
        const Tok &t = peek();
        if (t.k == Tok::NUM) {
            *out = Affine();
            out->c0 = t.v;
            ++k;
            return true;
        }
        if (t.k == Tok::IDENT) {
            for (auto &v : vars)
                if (v.first == t.s) {
                    *out = Affine();
                    out->v[v.second] = 1;
                    ++k;
                    return true;
                }
            int p = find_param(t.s, P_INT);
            if (p >= 0) {
                *out = Affine();
                out->p[p] = 1;
                ++k;
                return true;
            }
            if (find_param(t.s, P_ARRAY) >= 0)
                return fail("array '" + t.s + "' used inside an index (indirection is not expressible)");
            return fail("unknown name '" + t.s + "'");
        }
        if (is("(")) {
            ++k;
            if (!expr(out)) return false;
            return expect(")");
        }
        return fail("expected an index expression, found '" + t.s + "'");
    }

    bool unary(Affine *out) {
        if (is("-")) {
            ++k;
            if (!unary(out)) return false;
            scale(out, -1);
            return true;
        }
        if (is("+")) {
            ++k;
            return unary(out);
        }
        return primary(out);
    }

    static void scale(Affine *a, int64_t f) {
        a->c0 *= f;
        for (auto &x : a->v) x *= f;
        for (auto &x : a->p) x *= f;
    }
    static void addto(Affine *a, const Affine &b, int64_t sign) {
        a->c0 += sign * b.c0;
        for (int i = 0; i < NVAR; ++i) a->v[i] += sign * b.v[i];
        for (int i = 0; i < MAXPARAM; ++i) a->p[i] += sign * b.p[i];
    }
    static bool only_const(const Affine &a) {
        for (auto x : a.v)
            if (x) return false;
        return true;  // scalar parameters count as constants
    }

    bool term(Affine *out) {
        if (!unary(out)) return false;
        while (is("*")) {
            ++k;
            Affine r;
            if (!unary(&r)) return false;
            bool lc = out->is_const(), rc = r.is_const();
            if (lc) {
                int64_t f = out->c0;
                *out = r;
                scale(out, f);
            } else if (rc) {
                scale(out, r.c0);
            } else if (only_const(*out) && only_const(r)) {
                return fail("product of two scalar parameters is not supported");
            } else {
                return fail("index is not linear in the bound variables");
            }
        }
        return true;
    }

    bool expr(Affine *out) {
        if (!term(out)) return false;
        while (is("+") || is("-")) {
            int64_t sign = is("+") ? 1 : -1;
            ++k;
            Affine r;
            if (!term(&r)) return false;
            addto(out, r, sign);
        }
        return true;
    }

    bool index(IndexSpec *ix) {
        if (is(":")) {
            ++k;
            ix->has_lo = false;
            if (is(",") || is("]")) {
                ix->has_hi = false;
                return true;
            }
            return expr(&ix->hi);
        }
        if (!expr(&ix->lo)) return false;
        if (is(":")) {
            ++k;
            if (is(",") || is("]")) {
                ix->has_hi = false;
                return true;
            }
            return expr(&ix->hi);
        }
        ix->hi = ix->lo;
        return true;
    }

    bool binding(Annotation *an) {
        int kind;
        if (is("global")) kind = 0;
        else if (is("block")) kind = 1;
        else if (is("local")) kind = 2;
        else return fail("expected 'global', 'block' or 'local', found '" + peek().s + "'");
        if (an->nbound[kind] >= 0) return fail("binding kind bound twice");
        ++k;
        std::vector<std::string> names;
        if (is("[")) {
            ++k;
            for (;;) {
                if (peek().k != Tok::IDENT) return fail("expected a variable name");
                names.push_back(peek().s);
                ++k;
                if (is(",")) {
                    ++k;
                    continue;
                }
                if (!expect("]")) return false;
                break;
            }
        } else {
            if (peek().k != Tok::IDENT) return fail("expected a variable name");
            names.push_back(peek().s);
            ++k;
        }
        if (names.size() > 3) return fail("at most three axes can be bound");
        for (size_t i = 0; i < names.size(); ++i) {
            for (auto &v : vars)
                if (v.first == names[i]) return fail("variable '" + names[i] + "' bound twice");
            if (find_param(names[i], -1) >= 0)
                return fail("variable '" + names[i] + "' shadows a kernel parameter");
            vars.push_back({names[i], kind * 3 + (int)i});
        }
        an->nbound[kind] = (int)names.size();
        return true;
    }

    bool access(Annotation *an) {
        Access a;
        if (is("read")) a.mode = M_READ;
        else if (is("write")) a.mode = M_WRITE;
        else if (is("readwrite")) a.mode = M_RW;
        else if (is("reduce")) a.mode = M_REDUCE;
        else return fail("expected an access mode (read, write, readwrite, reduce), found '" + peek().s + "'");
        ++k;
        if (a.mode == M_REDUCE) {
            if (!expect("(")) return false;
            if (is("+")) a.op = R_ADD;
            else if (is("*")) a.op = R_MUL;
            else if (is("min")) a.op = R_MIN;
            else if (is("max")) a.op = R_MAX;
            else return fail("reduction operator must be +, *, min or max");
            ++k;
            if (!expect(")")) return false;
        }
        if (peek().k != Tok::IDENT) return fail("expected an array name");
        a.param = find_param(peek().s, P_ARRAY);
        if (a.param < 0) return fail("'" + peek().s + "' is not an array parameter of " + def->name);
        ++k;
        if (!expect("[")) return false;
        for (;;) {
            IndexSpec ix;
            if (!index(&ix)) return false;
            a.idx.push_back(ix);
            if (is(",")) {
                ++k;
                continue;
            }
            if (!expect("]")) return false;
            break;
        }
        an->acc.push_back(a);
        return true;
    }

    bool parse(Annotation *an) {
        if (!binding(an)) return false;
        while (is(",")) {
            ++k;
            if (!binding(an)) return false;
        }
        if (!expect("=>")) return false;
        if (!access(an)) return false;
        while (is(",")) {
            ++k;
            if (!access(an)) return false;
        }
        if (peek().k != Tok::END) return fail("trailing text '" + peek().s + "'");
        // every array parameter must be annotated; reduce cannot mix with
        // other modes on one array; index arity must match the rank
        for (int p = 0; p < def->nparam; ++p) {
            if (def->params[p].kind != P_ARRAY) continue;
            bool any = false, red = false, other = false;
            for (auto &a : an->acc) {
                if (a.param != p) continue;
                any = true;
                (a.mode == M_REDUCE ? red : other) = true;
                if ((int)a.idx.size() != def->params[p].ndim)
                    return fail(std::string("array '") + def->params[p].name + "' needs " +
                                std::to_string(def->params[p].ndim) + " indices");
            }
            if (!any) return fail(std::string("array parameter '") + def->params[p].name + "' is not annotated");
            if (red && other)
                return fail(std::string("array '") + def->params[p].name + "' mixes reduce with another mode");
        }
        int nb = -1;
        for (int kd = 0; kd < 3; ++kd) {
            if (an->nbound[kd] < 0) continue;
            if (nb >= 0 && an->nbound[kd] != nb) return fail("bindings bind different numbers of axes");
            nb = an->nbound[kd];
        }
        return true;
    }
};

}  // namespace

lt_status compile_annotation(Ctx *ctx, const KernelDef *def, const char *text,
                             std::shared_ptr<Annotation> *out) {
    if (!text) return set_err(ctx, LT_ERR_INVALID, "annotation is NULL");
    // definitions are told apart by address (user kernels may share names)
    char tag[32];
    snprintf(tag, sizeof tag, "%p\x1f", (const void *)def);
    std::string key = std::string(tag) + text;
    auto it = ctx->annot_cache.find(key);
    if (it != ctx->annot_cache.end()) {
        *out = it->second;
        return LT_OK;
    }
    std::string t(text);
    Lexer lx(t);
    Parser ps;
    ps.def = def;
    for (;;) {
        Tok tk;
        std::string e;
        if (!lx.next(&tk, &e)) return set_err(ctx, LT_ERR_PARSE, "annotation: %s", e.c_str());
        ps.toks.push_back(tk);
        if (tk.k == Tok::END) break;
    }
    auto an = std::make_shared<Annotation>();
    an->text = t;
    if (!ps.parse(an.get())) return set_err(ctx, LT_ERR_PARSE, "annotation: %s", ps.err.c_str());
    ctx->annot_cache[key] = an;
    *out = an;
    return LT_OK;
}

}  // namespace lt
