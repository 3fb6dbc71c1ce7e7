// Minimal JSON reader for model descriptions: objects, arrays, numbers,
// strings (with the common escapes), true/false/null.  Host only.
#pragma once
#include <cstdlib>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

namespace fn {
namespace json {

struct Value {
  enum Type { Null, Bool, Number, String, Array, Object } type = Null;
  bool b = false;
  double num = 0.0;
  std::string str;
  std::vector<Value> arr;
  std::map<std::string, Value> obj;

  bool has(const std::string& k) const { return type == Object && obj.count(k) != 0; }
  const Value& at(const std::string& k) const {
    if (type != Object) throw std::runtime_error("expected an object");
    auto it = obj.find(k);
    if (it == obj.end()) throw std::runtime_error("missing key \"" + k + "\"");
    return it->second;
  }
  double number() const {
    if (type != Number) throw std::runtime_error("expected a number");
    return num;
  }
  long integer() const {
    double v = number();
    if (v != static_cast<double>(static_cast<long>(v))) throw std::runtime_error("expected an integer");
    return static_cast<long>(v);
  }
  bool boolean() const {
    if (type != Bool) throw std::runtime_error("expected true/false");
    return b;
  }
  const std::string& string() const {
    if (type != String) throw std::runtime_error("expected a string");
    return str;
  }
  const std::vector<Value>& array() const {
    if (type != Array) throw std::runtime_error("expected an array");
    return arr;
  }
};

class Parser {
 public:
  explicit Parser(const char* s) : p_(s) {}
  Value parse() {
    Value v = value();
    ws();
    if (*p_) fail("trailing characters");
    return v;
  }

 private:
  const char* p_;
  [[noreturn]] void fail(const char* what) { throw std::runtime_error(std::string("JSON: ") + what); }
  void ws() {
    while (*p_ == ' ' || *p_ == '\n' || *p_ == '\t' || *p_ == '\r') ++p_;
  }
  bool lit(const char* w) {
    size_t n = 0;
    while (w[n]) ++n;
    for (size_t i = 0; i < n; ++i)
      if (p_[i] != w[i]) return false;
    p_ += n;
    return true;
  }
  Value value() {
    ws();
    Value v;
    if (*p_ == '{') {
      ++p_;
      v.type = Value::Object;
      ws();
      if (*p_ == '}') { ++p_; return v; }
      for (;;) {
        ws();
        if (*p_ != '"') fail("expected a key");
        std::string k = str();
        ws();
        if (*p_ != ':') fail("expected ':'");
        ++p_;
        v.obj[k] = value();
        ws();
        if (*p_ == ',') { ++p_; continue; }
        if (*p_ == '}') { ++p_; return v; }
        fail("expected ',' or '}'");
      }
    }
    if (*p_ == '[') {
      ++p_;
      v.type = Value::Array;
      ws();
      if (*p_ == ']') { ++p_; return v; }
      for (;;) {
        v.arr.push_back(value());
        ws();
        if (*p_ == ',') { ++p_; continue; }
        if (*p_ == ']') { ++p_; return v; }
        fail("expected ',' or ']'");
      }
    }
    if (*p_ == '"') {
      v.type = Value::String;
      v.str = str();
      return v;
    }
    if (lit("true")) { v.type = Value::Bool; v.b = true; return v; }
    if (lit("false")) { v.type = Value::Bool; v.b = false; return v; }
    if (lit("null")) { v.type = Value::Null; return v; }
    char* end = nullptr;
    double d = std::strtod(p_, &end);
    if (end == p_) fail("unexpected character");
    p_ = end;
    v.type = Value::Number;
    v.num = d;
    return v;
  }
  std::string str() {
    ++p_;  // opening quote
    std::string out;
    while (*p_ && *p_ != '"') {
      if (*p_ == '\\') {
        ++p_;
        switch (*p_) {
          case 'n': out += '\n'; break;
          case 't': out += '\t'; break;
          case '"': out += '"'; break;
          case '\\': out += '\\'; break;
          case '/': out += '/'; break;
          default: fail("unsupported escape");
        }
        ++p_;
      } else {
        out += *p_++;
      }
    }
    if (*p_ != '"') fail("unterminated string");
    ++p_;
    return out;
  }
};

inline Value parse(const char* s) { return Parser(s).parse(); }

}  // namespace json
}  // namespace fn
