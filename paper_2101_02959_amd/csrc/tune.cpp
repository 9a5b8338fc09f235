// Autotuner bookkeeping and its JSON cache (see tune.hpp).
#include "tune.hpp"

#include <cctype>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <memory>
#include <sstream>

namespace bdm {

namespace {

// Minimal JSON value and recursive-descent parser: objects, arrays,
// strings (with the standard escapes), numbers, true, false, null.
struct JVal {
    enum Kind { NUL, BOOL, NUM, STR, ARR, OBJ } kind = NUL;
    bool b = false;
    double num = 0;
    std::string str;
    std::vector<JVal> arr;
    std::vector<std::pair<std::string, JVal>> obj;
    const JVal* get(const std::string& k) const {
        for (const auto& kv : obj)
            if (kv.first == k) return &kv.second;
        return nullptr;
    }
};

struct Parser {
    const std::string& t;
    size_t i = 0;
    std::string err;
    explicit Parser(const std::string& s) : t(s) {}
    void ws() {
        while (i < t.size() && std::isspace((unsigned char)t[i])) ++i;
    }
    bool fail(const std::string& m) {
        if (err.empty()) err = m + " at offset " + std::to_string(i);
        return false;
    }
    bool lit(const char* w) {
        const size_t n = std::char_traits<char>::length(w);
        if (t.compare(i, n, w) != 0) return false;
        i += n;
        return true;
    }
    bool string(std::string& out) {
        if (i >= t.size() || t[i] != '"') return fail("expected string");
        ++i;
        out.clear();
        while (i < t.size() && t[i] != '"') {
            char c = t[i++];
            if (c == '\\') {
                if (i >= t.size()) return fail("bad escape");
                const char e = t[i++];
                switch (e) {
                    case '"': c = '"'; break;
                    case '\\': c = '\\'; break;
                    case '/': c = '/'; break;
                    case 'b': c = '\b'; break;
                    case 'f': c = '\f'; break;
                    case 'n': c = '\n'; break;
                    case 'r': c = '\r'; break;
                    case 't': c = '\t'; break;
                    case 'u': {
                        if (i + 4 > t.size()) return fail("bad unicode escape");
                        const unsigned code = (unsigned)std::strtoul(t.substr(i, 4).c_str(), nullptr, 16);
                        i += 4;
                        c = code < 128 ? (char)code : '?';
                        break;
                    }
                    default: return fail("bad escape");
                }
            }
            out.push_back(c);
        }
        if (i >= t.size()) return fail("unterminated string");
        ++i;
        return true;
    }
    bool value(JVal& v, int depth = 0) {
        if (depth > 32) return fail("nesting too deep");
        ws();
        if (i >= t.size()) return fail("unexpected end");
        const char c = t[i];
        if (c == '{') {
            ++i;
            v.kind = JVal::OBJ;
            ws();
            if (i < t.size() && t[i] == '}') { ++i; return true; }
            for (;;) {
                ws();
                std::string k;
                if (!string(k)) return false;
                ws();
                if (i >= t.size() || t[i] != ':') return fail("expected ':'");
                ++i;
                JVal x;
                if (!value(x, depth + 1)) return false;
                v.obj.emplace_back(k, std::move(x));
                ws();
                if (i < t.size() && t[i] == ',') { ++i; continue; }
                if (i < t.size() && t[i] == '}') { ++i; return true; }
                return fail("expected ',' or '}'");
            }
        }
        if (c == '[') {
            ++i;
            v.kind = JVal::ARR;
            ws();
            if (i < t.size() && t[i] == ']') { ++i; return true; }
            for (;;) {
                JVal x;
                if (!value(x, depth + 1)) return false;
                v.arr.push_back(std::move(x));
                ws();
                if (i < t.size() && t[i] == ',') { ++i; continue; }
                if (i < t.size() && t[i] == ']') { ++i; return true; }
                return fail("expected ',' or ']'");
            }
        }
        if (c == '"') {
            v.kind = JVal::STR;
            return string(v.str);
        }
        if (lit("true")) { v.kind = JVal::BOOL; v.b = true; return true; }
        if (lit("false")) { v.kind = JVal::BOOL; v.b = false; return true; }
        if (lit("null")) { v.kind = JVal::NUL; return true; }
        const char* p = t.c_str() + i;
        char* end = nullptr;
        const double d = std::strtod(p, &end);
        if (end == p) return fail("unexpected character");
        i += (size_t)(end - p);
        v.kind = JVal::NUM;
        v.num = d;
        return true;
    }
};

std::string quote(const std::string& s) {
    std::string o = "\"";
    for (const char c : s) {
        if (c == '"' || c == '\\') {
            o.push_back('\\');
            o.push_back(c);
        } else if ((unsigned char)c < 0x20) {
            char buf[8];
            std::snprintf(buf, sizeof buf, "\\u%04x", (unsigned)c);
            o += buf;
        } else {
            o.push_back(c);
        }
    }
    return o + "\"";
}

std::string num(double x) {
    if (!std::isfinite(x)) return "-1";
    char buf[32];
    std::snprintf(buf, sizeof buf, "%.6g", x);
    return buf;
}

}  // namespace

std::string tune_to_json(const std::vector<TuneEntry>& e) {
    std::ostringstream o;
    o << "{\"format\": \"bidomain-tune-1\", \"entries\": [";
    for (size_t k = 0; k < e.size(); ++k) {
        const TuneEntry& x = e[k];
        o << (k ? ", " : "") << "{\"device\": " << quote(x.device) << ", \"family\": " << quote(x.family)
          << ", \"class\": " << quote(x.cls) << ", \"choice\": " << x.choice << ", \"ms\": [";
        for (size_t j = 0; j < x.ms.size(); ++j) o << (j ? ", " : "") << num(x.ms[j]);
        o << "], \"cached\": " << (x.cached ? "true" : "false") << "}";
    }
    o << "]}";
    return o.str();
}

std::string tune_from_json(const std::string& text, std::vector<TuneEntry>& out) {
    Parser p(text);
    JVal root;
    if (!p.value(root)) return "tune cache: " + p.err;
    p.ws();
    if (p.i != text.size()) return "tune cache: trailing characters";
    const JVal* fmt = root.kind == JVal::OBJ ? root.get("format") : nullptr;
    if (!fmt || fmt->kind != JVal::STR || fmt->str != "bidomain-tune-1") return "tune cache: unknown format";
    const JVal* ent = root.get("entries");
    if (!ent || ent->kind != JVal::ARR) return "tune cache: no entries array";
    std::vector<TuneEntry> res;
    for (const JVal& v : ent->arr) {
        if (v.kind != JVal::OBJ) return "tune cache: entry is not an object";
        const JVal *d = v.get("device"), *f = v.get("family"), *c = v.get("class"), *ch = v.get("choice"),
                   *ms = v.get("ms");
        if (!d || !f || !c || !ch || d->kind != JVal::STR || f->kind != JVal::STR || c->kind != JVal::STR ||
            ch->kind != JVal::NUM || ch->num < 0 || ch->num != std::floor(ch->num))
            return "tune cache: malformed entry";
        TuneEntry e;
        e.device = d->str;
        e.family = f->str;
        e.cls = c->str;
        e.choice = (int)ch->num;
        if (ms && ms->kind == JVal::ARR)
            for (const JVal& m : ms->arr)
                if (m.kind == JVal::NUM) e.ms.push_back(m.num);
        e.cached = true;
        res.push_back(std::move(e));
    }
    out = std::move(res);
    return "";
}

std::string Tuner::load(const std::string& path) {
    std::ifstream f(path);
    if (!f) return "";   // no cache yet
    std::stringstream ss;
    ss << f.rdbuf();
    std::vector<TuneEntry> e;
    const std::string err = tune_from_json(ss.str(), e);
    if (!err.empty()) return err;
    entries = std::move(e);
    return "";
}

std::string Tuner::save(const std::string& path) const {
    std::vector<TuneEntry> e = entries;
    for (auto& x : e) x.cached = false;
    const std::string tmp = path + ".tmp" + std::to_string((long)std::rand());
    {
        std::ofstream f(tmp);
        if (!f) return "cannot write " + tmp;
        f << tune_to_json(e) << "\n";
        if (!f) return "cannot write " + tmp;
    }
    if (std::rename(tmp.c_str(), path.c_str()) != 0) {
        std::remove(tmp.c_str());
        return "cannot rename the tune cache to " + path;
    }
    return "";
}

int Tuner::pick(const std::string& family, const std::string& cls, int nvar,
                const std::function<double(int)>& time_ms) {
    for (size_t k = 0; k < entries.size(); ++k) {
        const TuneEntry& e = entries[k];
        if (e.device == device && e.family == family && e.cls == cls && e.choice < nvar) {
            used.push_back((int)k);
            return e.choice;
        }
    }
    TuneEntry e;
    e.device = device;
    e.family = family;
    e.cls = cls;
    e.ms.assign(nvar, -1.0);
    int best = 0;
    double tbest = -1.0;
    for (int v = 0; v < nvar; ++v) {
        const double t = time_ms(v);
        e.ms[v] = t;
        if (t >= 0 && (tbest < 0 || t < tbest)) {
            tbest = t;
            best = v;
        }
    }
    // Variants within 1% of the fastest are a tie (run-to-run timing noise
    // is about that): the lowest-numbered of them is taken, so repeated
    // tunings of one build settle on the same variant.
    for (int v = 0; v < best; ++v)
        if (e.ms[v] >= 0 && e.ms[v] <= 1.01 * tbest) {
            best = v;
            break;
        }
    e.choice = best;
    entries.push_back(std::move(e));
    used.push_back((int)entries.size() - 1);
    dirty = true;
    return best;
}

std::string Tuner::report() const {
    std::vector<TuneEntry> e;
    for (const int k : used) e.push_back(entries[k]);
    return tune_to_json(e);
}

}  // namespace bdm
